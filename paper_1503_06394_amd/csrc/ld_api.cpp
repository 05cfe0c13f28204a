// Host planner and C-ABI entry points of liblogdet_cheb (see include/logdet_cheb.h).
//
// The planner validates arguments, computes the Chebyshev coefficients of eq. (1) in
// FP64, folds the affine map of Section 4.1 into the step scalars
//     alpha = 4 / (b - a),  beta = -2 (a + b) / (b - a)   (2 At = alpha B + beta I),
// picks a kernel shape (autotuned once per matrix signature), carves the workspace, and
// enqueues the recurrence steps of Algorithm 1 (or Algorithm 2, the adjoint, or the
// batch) on the caller's stream.  Per-probe moments come back to the host, where the
// estimate Gamma = (1/M) sum_j sum_k c_k mu[j][k] is formed in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../../include/logdet_cheb.h"
#include "ld_internal.h"

using namespace ld;

namespace {

thread_local char g_err[512] = "";

// Records the message for ld_last_error (never allocates, never throws) and returns `code`.
int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

// Runs an entry point's body so that no C++ exception (host allocation failure in a std::vector,
// std::map, ...) crosses the C ABI.  Status-returning entry points then return LD_ENOMEM or
// LD_EINVAL; ld_workspace_bytes returns 0.  The message is left for ld_last_error.
template <typename R, typename F>
R guarded(F&& body) noexcept {
  int code;
  try {
    return body();
  } catch (const std::bad_alloc&) {
    code = fail(LD_ENOMEM, "host memory allocation failed");
  } catch (const std::exception& e) {
    code = fail(LD_EINVAL, "internal error: %s", e.what());
  } catch (...) {
    code = fail(LD_EINVAL, "internal error");
  }
  return std::is_same<R, int>::value ? (R)code : (R)0;
}

int fail_hip(hipError_t e, const char* what) {
  return fail(LD_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define LD_HIP(call)                               \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return fail_hip(e_, #call); \
  } while (0)

constexpr size_t kAlign = 256;
constexpr size_t kDotScratch = 512;  // blocks of the FP64 dot-product partials
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Sequential carve of a device workspace (first pass with base == nullptr sizes it).
struct Carve {
  char* base = nullptr;
  size_t off = 0;
  void* take(size_t bytes) {
    off = align_up(off);
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

// Device buffers the library reuses across calls that bring no workspace of their own: per device,
// at most kPoolKeep idle buffers are kept (until ld_clear_cache); a call takes the smallest idle one
// that is large enough, or allocates a new one.  Nested and concurrent calls take different buffers.
struct PoolBuf {
  void* ptr;
  size_t bytes;
};
std::mutex g_pool_mu;
std::map<int, std::vector<PoolBuf>> g_pool;  // device -> idle buffers
constexpr size_t kPoolKeep = 4;

void pool_release_all() {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  for (auto& kv : g_pool)
    for (auto& b : kv.second) (void)hipFree(b.ptr);
  g_pool.clear();
}

// Workspace: the caller's, or a pooled buffer returned to the pool on scope exit (after the stream
// it served has drained, so no later call can overlap work still reading it).
struct Workspace {
  void* ptr = nullptr;
  size_t bytes = 0;
  int device = -1;
  bool pooled = false;
  hipStream_t stream = nullptr;
  ~Workspace() {
    if (!pooled) return;
    (void)hipStreamSynchronize(stream);
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto& idle = g_pool[device];
    idle.push_back(PoolBuf{ptr, bytes});
    if (idle.size() > kPoolKeep) {  // drop the smallest
      auto it = std::min_element(idle.begin(), idle.end(),
                                 [](const PoolBuf& x, const PoolBuf& y) { return x.bytes < y.bytes; });
      (void)hipFree(it->ptr);
      idle.erase(it);
    }
  }
};

// Bytes of the idle pooled buffers on the current device: memory the library can reuse at once.
size_t pool_idle_bytes() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  size_t sum = 0;
  auto it = g_pool.find(dev);
  if (it != g_pool.end())
    for (const PoolBuf& b : it->second) sum += b.bytes;
  return sum;
}

int get_workspace(const ld_opts* opt, size_t need, hipStream_t s, Workspace& ws) {
  ws.stream = s;
  if (opt && opt->workspace) {
    if (reinterpret_cast<uintptr_t>(opt->workspace) % kAlign)
      return fail(LD_EINVAL, "workspace must be %zu-byte aligned", kAlign);
    if (opt->workspace_bytes < need)
      return fail(LD_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu bytes needed", opt->workspace_bytes,
                  need);
    ws.ptr = opt->workspace;
    return LD_OK;
  }
  if (need == 0) return LD_OK;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto& idle = g_pool[dev];
    auto best = idle.end();
    for (auto it = idle.begin(); it != idle.end(); ++it)
      if (it->bytes >= need && (best == idle.end() || it->bytes < best->bytes)) best = it;
    if (best != idle.end()) {
      ws.ptr = best->ptr;
      ws.bytes = best->bytes;
      idle.erase(best);
    }
  }
  if (!ws.ptr) {
    e = hipMalloc(&ws.ptr, need);
    if (e != hipSuccess) {
      pool_release_all();  // idle buffers may be what stands in the way
      e = hipMalloc(&ws.ptr, need);
    }
    if (e != hipSuccess) return fail(LD_ENOMEM, "hipMalloc(%zu): %s", need, hipGetErrorString(e));
    ws.bytes = need;
  }
  ws.device = dev;
  ws.pooled = true;
  return LD_OK;
}

int valt_of(int32_t dtype) {
  switch (dtype) {
    case LD_F64: return VAL_F64;
    case LD_F32: return VAL_F32;
    case LD_BF16: return VAL_BF16;
    default: return -1;
  }
}

size_t val_bytes(int valt) { return valt == VAL_F64 ? 8 : (valt == VAL_F32 ? 4 : 2); }

int check_csr(const ld_csr* B, const char* name) {
  if (!B) return fail(LD_EINVAL, "%s is NULL", name);
  if (B->rows < 0 || B->rows != B->cols) return fail(LD_EINVAL, "%s must be square (rows=%lld cols=%lld)", name,
                                                     (long long)B->rows, (long long)B->cols);
  if (B->nnz < 0 || (B->rows > 0 && B->nnz > B->rows * B->cols))
    return fail(LD_EINVAL, "%s has invalid nnz %lld", name, (long long)B->nnz);
  if (B->rows > 0 && !B->row_ptr) return fail(LD_EINVAL, "%s->row_ptr is NULL", name);
  if (B->nnz > 0 && (!B->col_idx || !B->values)) return fail(LD_EINVAL, "%s has NULL col_idx or values", name);
  if (B->rows > (int64_t)0x7FFFFFFF) return fail(LD_EINVAL, "%s has more than 2^31-1 rows", name);
  if (valt_of(B->dtype) < 0) return fail(LD_EDTYPE, "%s has unknown dtype %d", name, B->dtype);
  if (B->reserved != 0) return fail(LD_EINVAL, "%s->reserved must be 0", name);
  if (!std::isfinite(B->diag_shift)) return fail(LD_EINVAL, "%s->diag_shift is not finite", name);
  return LD_OK;
}

int check_common(double a, double b, int n, int M) {
  if (!std::isfinite(a) || !std::isfinite(b) || !(a > 0.0) || !(b > a))
    return fail(LD_EINVAL, "bounds must satisfy 0 < a < b (finite); got a=%g b=%g", a, b);
  if (n < 0 || n > 100000) return fail(LD_EINVAL, "degree n=%d out of range [0, 100000]", n);
  if (M < 1 || M > 4096) return fail(LD_EINVAL, "probe count M=%d out of range [1, 4096]", M);
  return LD_OK;
}

// eq. (1): interpolant of f(x) = log(((b - a) x + (a + b)) / 2) at x_k = cos(pi (k + 1/2) / (n + 1)),
// using T_i(cos t) = cos(i t).
std::vector<double> cheb_coeffs(double a, double b, int n) {
  const double pi = 3.14159265358979323846;
  std::vector<double> fx(n + 1), th(n + 1), c(n + 1);
  for (int k = 0; k <= n; ++k) {
    th[k] = pi * (k + 0.5) / (n + 1);
    fx[k] = std::log(((b - a) * std::cos(th[k]) + (a + b)) / 2.0);
  }
  for (int i = 0; i <= n; ++i) {
    double s = 0.0;
    for (int k = 0; k <= n; ++k) s += fx[k] * std::cos(i * th[k]);
    c[i] = (i == 0 ? 1.0 : 2.0) / (n + 1) * s;
  }
  return c;
}

// Lemma 7: 20 d log(2 (1/delta - 1)) / ((K - 1) K^n), delta = a / (a + b).
double lemma_bound(double a, double b, int n, int64_t d) {
  const double delta = a / (a + b);
  const double K = (std::sqrt(2.0 - delta) + std::sqrt(delta)) / (std::sqrt(2.0 - delta) - std::sqrt(delta));
  return 20.0 * (double)d * std::log(2.0 * (1.0 / delta - 1.0)) / ((K - 1.0) * std::pow(K, n));
}

// ------------------------------------------------------------------------------------
// kernel shape planning and autotuning
// ------------------------------------------------------------------------------------

// Lane layout for M probes: VPL consecutive probes per lane (a 16-byte vector where M
// allows), LPR = 2^lpr_log2 lanes per row.  probe_tile > 0 narrows the group so that one
// pass over the matrix covers only that many probes; the launch then walks the probe tiles
// one after another (blockIdx.y), which keeps the live slice of W_k small enough to stay in
// the Infinity Cache.
Shape base_shape(int vec_f64, int M, int probe_tile = 0) {
  Shape sh{};
  if (!vec_f64)
    sh.vpl = (M % 4 == 0) ? 4 : ((M % 2 == 0) ? 2 : 1);
  else
    sh.vpl = (M % 2 == 0) ? 2 : 1;
  const int want = probe_tile > 0 ? std::min(probe_tile, M) : M;
  int lanes = (want + sh.vpl - 1) / sh.vpl;
  int lg = 0;
  while ((1 << lg) < lanes && lg < 6) ++lg;
  sh.lpr_log2 = lg;
  const int tile_probes = (1 << lg) * sh.vpl;
  sh.probe_tiles = (M + tile_probes - 1) / tile_probes;
  return sh;
}

// Probe-tile layouts the autotuner tries: the full block and up to two narrower ones
// (at least 16 probes and 4 lanes per row).
std::vector<Shape> shape_candidates(int vec_f64, int M) {
  std::vector<Shape> out;
  const Shape full = base_shape(vec_f64, M);
  out.push_back(full);
  for (int drop = 1; drop <= 2; ++drop) {
    const int lg = full.lpr_log2 - drop;
    if (lg < 2 || ((1 << lg) * full.vpl) < 16) break;
    out.push_back(base_shape(vec_f64, M, (1 << lg) * full.vpl));
  }
  return out;
}

int rows_per_iter(const Shape& sh) { return 4 * (64 >> sh.lpr_log2); }

// Largest tile height whose CSR slice fits the LDS staging buffer on average (with a
// margin for rows longer than the mean), as a multiple of the rows one pass covers.
int staged_tile_cap(const Shape& sh, int64_t d, int64_t nnz) {
  const int rpi = rows_per_iter(sh);
  const double per_row = d > 0 ? std::max(1.0, (double)nnz / (double)d) : 1.0;
  int64_t rows = (int64_t)(0.8 * kStageNnz / per_row);
  rows = std::min<int64_t>(rows, kStageRows);
  rows = rows / rpi * rpi;
  return (int)std::max<int64_t>(rows, rpi);
}

// Default tile height: as tall as the LDS slice allows, but short enough that the matrix
// spreads over at least ~1024 workgroups.
Shape with_tile(Shape sh, int64_t d, int64_t nnz, int tile_override) {
  const int rpi = rows_per_iter(sh);
  if (tile_override > 0) {
    sh.tile_rows = (tile_override + rpi - 1) / rpi * rpi;
    return sh;
  }
  const int64_t spread = std::max<int64_t>(rpi, d / 1024 / rpi * rpi);
  sh.tile_rows = (int)std::min<int64_t>(staged_tile_cap(sh, d, nnz), spread);
  return sh;
}

// Tile heights the autotuner tries: the staging cap and two smaller heights.
std::vector<int> tile_candidates(const Shape& sh, int64_t d, int64_t nnz) {
  const int rpi = rows_per_iter(sh);
  const int cap = with_tile(sh, d, nnz, 0).tile_rows;
  std::vector<int> c;
  for (int div : {1, 2, 4}) {
    const int r = std::max(rpi, cap / div / rpi * rpi);
    if (std::find(c.begin(), c.end(), r) == c.end()) c.push_back(r);
  }
  return c;
}


struct TuneKey {
  int vec, valt, M, mode;
  int64_t d, nnz;
  bool operator<(const TuneKey& o) const {
    return std::tie(vec, valt, M, mode, d, nnz) < std::tie(o.vec, o.valt, o.M, o.mode, o.d, o.nnz);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, Shape> g_tune;

// LD_GRAD_SYM=0 forces the two-gather adjoint even for symmetric patterns (for testing).
bool sym_enabled() {
  const char* e = std::getenv("LD_GRAD_SYM");
  return !(e && e[0] == '0');
}

// Form of the paired adjoint: LD_GRAD_FORM=shifted or =explicit forces one (for tests); otherwise
// -1 (chosen from the pattern).
int grad_form_override() {
  const char* e = std::getenv("LD_GRAD_FORM");
  if (!e) return -1;
  if (std::strcmp(e, "shifted") == 0) return 1;
  if (std::strcmp(e, "explicit") == 0) return 0;
  return -1;
}

// LD_AUTOTUNE=0 keeps the default tile height and probe layout (no timing of candidates).
bool autotune_enabled() {
  const char* e = std::getenv("LD_AUTOTUNE");
  return !(e && e[0] == '0');
}

// Time the general recurrence step (k >= 2 form) for each candidate probe-tile layout and
// tile height on the caller's data and return the fastest.  Buffers are scratch; their
// contents do not matter for timing.
Shape autotune(const ld_csr* B, const std::vector<Shape>& shapes, int vec_f64, int valt, int M, int mu_mode,
               void* bufA, void* bufB, double* part, hipStream_t s) {
  Shape best_sh = shapes[0];
  best_sh.tile_rows = 0;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return best_sh;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return best_sh;
  }
  float best = 1e30f;
  for (const Shape& base : shapes) {
    for (int rows : tile_candidates(base, B->rows, B->nnz)) {
      Shape sh = base;
      sh.tile_rows = rows;
      StepLaunch L{};
      L.nmat = 1;
      L.ntiles = (B->rows + sh.tile_rows - 1) / sh.tile_rows;
      L.tile_rows = sh.tile_rows;
      L.M = M;
      L.shape = sh;
      StepDesc& D = L.d0;
      D.row_ptr = B->row_ptr;
      D.col = B->col_idx;
      D.val = B->values;
      D.G = bufA;
      D.P = bufB;
      D.out = bufB;
      D.ag = 1.0;
      D.bd = 0.0;
      D.cp = -1.0;
      D.d = B->rows;
      D.mu_part = part;
      D.mu_part2 = part;  // timing only: both partial slots may overlap
      D.active = 1;
      float tot = 0.f;
      bool ok = true;
      for (int rep = 0; rep < 4 && ok; ++rep) {
        ok = hipEventRecord(e0, s) == hipSuccess &&
             launch_step(L, vec_f64, valt, SRC_BUF, SRC_SAME, SRC_BUF, mu_mode, s) == hipSuccess &&
             hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.f;
        if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && rep > 0) tot += ms;
      }
      if (ok && tot < best) {
        best = tot;
        best_sh = sh;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best_sh;
}

// ------------------------------------------------------------------------------------
// step timing (HIP events on the launch stream)
// ------------------------------------------------------------------------------------

// Interval kinds recorded by StepTimer::mark: what ran since the previous mark.
enum : int { T_OTHER = 0, T_STEP = 1, T_ADJ = 2 };

struct StepTimer {
  bool on = false;
  hipStream_t s = nullptr;
  std::vector<hipEvent_t> ev;
  std::vector<int> kind;  // kind of interval i (between events i and i+1)
  ~StepTimer() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
  hipError_t mark(int interval_kind) {
    if (!on) return hipSuccess;
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    ev.push_back(e);
    if (ev.size() > 1) kind.push_back(interval_kind);
    return hipEventRecord(e, s);
  }
  void report(ld_result* out) {
    out->kernel_ms = 0.0;
    out->kernel_launches = 0;
    out->adjoint_ms = 0.0;
    out->adjoint_launches = 0;
    if (!on) return;
    for (size_t i = 0; i + 1 < ev.size(); ++i) {
      if (kind[i] == T_OTHER) continue;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) != hipSuccess) continue;
      if (kind[i] == T_STEP) {
        out->kernel_ms += ms;
        out->kernel_launches += 1;
      } else {
        out->adjoint_ms += ms;
        out->adjoint_launches += 1;
      }
    }
  }
};

// Combine FP64 moments into the estimate (host, FP64).  mu is M x (n+1) row-major.
void combine(const std::vector<double>& mu, const std::vector<double>& c, int n, int M, int64_t d, double half,
             ld_result* out, const ld_opts* opt) {
  std::vector<double> sj(M);
  uint32_t flags = 0;
  const double lim = (double)d * (1.0 + 1e-6);
  for (int j = 0; j < M; ++j) {
    double s = 0.0;
    for (int k = 0; k <= n; ++k) {
      const double m = mu[(size_t)j * (n + 1) + k];
      if (!(std::fabs(m) <= lim)) flags |= 1u;
      s += c[k] * m;
    }
    sj[j] = s * half;
  }
  double mean = 0.0;
  for (int j = 0; j < M; ++j) mean += sj[j];
  mean /= M;
  double var = 0.0;
  for (int j = 0; j < M; ++j) var += (sj[j] - mean) * (sj[j] - mean);
  out->logdet = mean;
  out->std_err = M > 1 ? std::sqrt(var / (M - 1) / M) : NAN;
  out->flags = flags;
  out->n = n;
  out->M = M;
  if (opt && opt->moments_out) std::memcpy(opt->moments_out, mu.data(), sizeof(double) * mu.size());
  if (opt && opt->probe_out) std::memcpy(opt->probe_out, sj.data(), sizeof(double) * M);
}

int vec_f64_of(const ld_opts* opt, int valt) {
  if (!opt || opt->vec_f64 == 0) return valt == VAL_F64 ? 1 : 0;
  return opt->vec_f64 == 1 ? 1 : 0;
}

// Product identities (default) or one sparse product per degree.
bool use_pairs(const ld_opts* opt) { return !(opt && opt->plain_recurrence); }

// Sparse products per probe block: n, or ceil(n/2) with the product identities.
int steps_for(int n, bool pair) { return pair ? (n + 1) / 2 : n; }

// Partial rows written: one per step, or two per step (W_k^T W_{k+1}, W_{k+1}^T W_{k+1}).
int partial_rows(int n, bool pair) { return pair ? 2 * steps_for(n, pair) : n; }

// Moments mu[j][0..n] (M x (n+1)) from the reduced partial rows red[j][0..nrows).
// Plain: row k holds v^T W_{k+1}.  Pairs: row 2k holds a_k = W_k^T W_{k+1}, row 2k+1 holds
// b_k = W_{k+1}^T W_{k+1} (W_0 = v); with T_{2k+2} = 2 T_{k+1}^2 - T_0 and
// T_{2k+1} = 2 T_{k+1} T_k - T_1 for symmetric At:
//   mu_1 = a_0,  mu_{2k+2} = 2 b_k - d,  mu_{2k+1} = 2 a_k - mu_1 (k >= 1).
void assemble_moments(const std::vector<double>& red, int nrows, bool pair, int n, int M, int64_t d,
                      std::vector<double>& mu) {
  for (int j = 0; j < M; ++j) {
    double* m = &mu[(size_t)j * (n + 1)];
    const double* r = red.data() + (size_t)j * std::max(nrows, 1);
    m[0] = (double)d;  // v^T v = d for Rademacher probes
    if (!pair) {
      for (int k = 1; k <= n; ++k) m[k] = r[k - 1];
      continue;
    }
    if (n >= 1) m[1] = r[0];
    for (int k = 0; 2 * k + 1 < nrows; ++k) {
      if (2 * k + 2 <= n) m[2 * k + 2] = 2.0 * r[2 * k + 1] - (double)d;
      if (k >= 1 && 2 * k + 1 <= n) m[2 * k + 1] = 2.0 * r[2 * k] - m[1];
    }
  }
}

// ------------------------------------------------------------------------------------
// Algorithm 1 / Algorithm 2 forward driver
// ------------------------------------------------------------------------------------

struct FwdPlan {
  Shape sh;
  int64_t ntiles;
  size_t vb;
};

FwdPlan plan_fwd(const ld_csr* B, int vec_f64, int M, const ld_opts* opt) {
  FwdPlan p;
  p.sh = with_tile(base_shape(vec_f64, M, opt ? opt->probe_tile : 0), B->rows, B->nnz, opt ? opt->tile : 0);
  p.ntiles = B->rows > 0 ? (B->rows + p.sh.tile_rows - 1) / p.sh.tile_rows : 0;
  p.vb = vec_f64 ? 8 : 4;
  return p;
}

// Largest number of row tiles any shape the planner or the autotuner may pick produces.
int64_t max_tiles(const ld_csr* B, int vec_f64, int M, const ld_opts* opt) {
  if (B->rows <= 0) return 0;
  if (opt && opt->tile > 0) return plan_fwd(B, vec_f64, M, opt).ntiles;
  std::vector<Shape> shapes = (opt && opt->probe_tile > 0)
                                  ? std::vector<Shape>{base_shape(vec_f64, M, opt->probe_tile)}
                                  : shape_candidates(vec_f64, M);
  int min_rows = 1 << 30;
  for (const Shape& sh : shapes)
    for (int r : tile_candidates(sh, B->rows, B->nnz)) min_rows = std::min(min_rows, r);
  return (B->rows + min_rows - 1) / min_rows;
}

// Probe block the forward actually runs.  Some block widths run slower than a wider one (forward
// times on random patterns at d = 10^6 and 3 10^6):
//  * under 16 probes, rows that are not a whole number of 64-byte segments: widened to the lane
//    group the shape gives them anyway (LPR lanes x VPL probes), so every lane issues an aligned
//    vector load and no gathered row straddles a segment (10 probes take longer per step than 16);
//  * rows held by a single 16-byte lane (FP32 M = 3, 4; FP64 M = 2): widened to two lanes;
//  * FP32 rows that straddle 128-byte lines (17..31 and 49..63 probes): widened to the next whole
//    line (24 probes take 7.6 ms, 32 take 6.3 ms; 56 take 13.1 ms, 64 take 11.8 ms).
// Probes are indexed, so the first M are the same probes; the estimate drops the rest.
int padded_probes(int M, int vec_f64, const ld_opts* opt) {
  if (opt && opt->probe_tile > 0) return M;
  if (!vec_f64) {
    if (M == 3 || M == 4) return 8;
    if (M > 16 && M < 32) return 32;
    if (M > 48 && M < 64) return 64;
  } else if (M == 2) {
    return 4;
  }
  const int vb = vec_f64 ? 8 : 4;
  if (M >= 16 || (M * vb) % 64 == 0) return M;
  const Shape sh = base_shape(vec_f64, M);
  const int width = (1 << sh.lpr_log2) * sh.vpl;
  return (sh.probe_tiles == 1 && width <= 16) ? width : M;
}

size_t fwd_workspace(const ld_csr* B, int n, int M, int vec_f64, bool ns, const ld_opts* opt) {
  M = padded_probes(M, vec_f64, opt);
  const size_t vb = vec_f64 ? 8 : 4;
  const int64_t tiles = max_tiles(B, vec_f64, M, opt);
  Carve c;
  const size_t vecb = (size_t)B->rows * M * vb;
  c.take(vecb);  // A
  c.take(vecb);  // B
  if (ns) {
    c.take(vecb);                                   // T
    c.take((size_t)(B->rows + 1) * 8);              // Ct row_ptr
    c.take((size_t)B->nnz * 4);                     // Ct col
    c.take((size_t)B->nnz * val_bytes(valt_of(B->dtype)));
    c.take((size_t)B->rows * 8);                    // cursor
    c.take(transpose_scratch_bytes(B->rows));
  }
  const int rows = std::max(partial_rows(n, use_pairs(opt)), 1);
  c.take((size_t)rows * tiles * M * 8);  // per-tile partials
  c.take((size_t)M * rows * 8);          // reduced partials
  c.take(reduce_scratch_bytes(rows, M));  // reduction stage 1
  c.take(256);                            // pattern hash (staged steps)
  return align_up(c.off);
}


// ------------------------------------------------------------------------------------
// Taylor-series comparator: W_k = A W_{k-1}, A = I - (B + shift I)/(a + b), moments v^T A^k v
// ------------------------------------------------------------------------------------

size_t taylor_workspace(const ld_csr* B, int n, int M, int vec_f64, const ld_opts* opt) {
  const size_t vb = vec_f64 ? 8 : 4;
  const int64_t tiles = max_tiles(B, vec_f64, M, opt);
  const int rows = std::max(n, 1);
  Carve c;
  c.take((size_t)B->rows * M * vb);
  c.take((size_t)B->rows * M * vb);
  c.take((size_t)rows * tiles * M * 8);
  c.take((size_t)M * rows * 8);
  c.take(reduce_scratch_bytes(rows, M));
  c.take(256);  // pattern hash (staged steps)
  return align_up(c.off);
}


}  // namespace

// ======================================================================================
// gradient
// ======================================================================================

namespace {

// Checkpoint plan of the gradient.  The forward produces W_1..W_m (m = n plain, ceil(n/2)
// with the product identities).  The adjoint starts from y_top (top = n plain, m pairs) and
// steps j = top-1 .. 1; step j needs W_j and, with pairs, W_{j-1} and W_{j+1} for its seed.
// Steps are grouped in segments of s = ceil(sqrt(top)) consecutive j; segment q (j in
// [lo, hi]) keeps the pair (W_{lo-1}, W_lo) from the forward pass and recomputes
// W_{lo+1}..W_hi; W_{hi+1} is the next segment's checkpoint (or W_top).
struct GradPlan {
  bool pair;
  int m, top, s, nseg;
  std::vector<int> lo, hi;   // per segment
  std::vector<int> slot_of;  // W_k -> checkpoint slot or -1, k = 0..m
  int nslots;
  int nseg_buf;              // recomputation scratch blocks (also the forward's rolling pair)
};

GradPlan plan_grad(int n, bool pair, int stride) {
  GradPlan g;
  g.pair = pair;
  g.m = steps_for(n, pair);
  g.top = pair ? g.m : n;
  const int nsteps = std::max(g.top - 1, 0);  // adjoint steps j = top-1 .. 1
  g.s = stride > 0 ? stride : (int)std::ceil(std::sqrt((double)std::max(nsteps, 1)));
  if (g.s < 1) g.s = 1;
  g.nseg = nsteps > 0 ? (nsteps - 1) / g.s + 1 : 0;
  g.slot_of.assign(g.m + 2, -1);
  g.nslots = 0;
  auto keep = [&](int k) {
    if (k >= 1 && k <= g.m && g.slot_of[k] < 0) g.slot_of[k] = g.nslots++;
  };
  for (int q = 0; q < g.nseg; ++q) {
    g.lo.push_back(1 + q * g.s);
    g.hi.push_back(std::min(1 + (q + 1) * g.s - 1, g.top - 1));
    keep(g.lo[q] - 1);
    keep(g.lo[q]);
  }
  if (pair) {  // the seed of y_top and the last step's W_{hi+1}
    keep(g.top - 1);
    keep(g.top);
  }
  g.nseg_buf = std::max(g.s - 1, 2);
  return g;
}

// Kernel shape of a gradient pass: the pass's whole probe block in one lane group (the adjoint
// reduces across it), the caller's tile height or the default one.
Shape grad_shape(const ld_csr* B, int M, int vec_f64, const ld_opts* opt) {
  return with_tile(base_shape(vec_f64, M), B->rows, B->nnz, opt ? opt->tile : 0);
}

// Tile of the plane-major order (the default tile height unless the caller set one): a power-of-two
// number of row passes no taller than the default tile, which divides the planes of lattices whose
// sides are multiples of a power of two.
Shape plane_shape(const Shape& def, const ld_opts* opt) {
  Shape sh = def;
  if (opt && opt->tile > 0) return sh;
  const int rpi = rows_per_iter(sh);
  int r = rpi;
  while (2 * r <= sh.tile_rows) r *= 2;
  sh.tile_rows = r;
  return sh;
}

// Probes per gradient pass.  Wider blocks would hold one row per wave, where the adjoint's
// cross-lane reductions cost more than a second pass over the matrix (FP32: 256 probes in one
// pass take 13 % longer than two passes of 128).  A chunk size that is a multiple of 64 keeps
// every pass's probes on whole words of the probe hash.
struct GradChunks {
  int size, count, last;  // probes per full pass, passes, probes in the last pass
};

GradChunks grad_chunks(int M, int vec_f64) {
  const int cap = vec_f64 ? 64 : 128;
  GradChunks c;
  c.size = std::min(M, cap);
  c.count = (M + c.size - 1) / c.size;
  c.last = M - (c.count - 1) * c.size;
  return c;
}

// Seed under which a pass's local probe j is global probe probe0 + j, for probe0 a multiple of
// 64.  The counter hash takes the SplitMix64 state seed + (ctr + 1) * gamma with
// ctr = (row << 16) | (probe >> 6) (gamma = 0x9E3779B97F4A7C15, the generator's increment);
// fewer than 2^16 words per row means the | is a +, so moving the probe-word index by probe0/64
// is the same as adding (probe0/64) * gamma to the seed (mod 2^64).
uint64_t pass_seed(uint64_t seed, int probe0) {
  return seed + (uint64_t)(probe0 >> 6) * 0x9E3779B97F4A7C15ull;
}

int64_t tiles_of(const ld_csr* B, const Shape& sh) {
  return B->rows > 0 ? (B->rows + sh.tile_rows - 1) / sh.tile_rows : 0;
}

// Tiles a gradient pass of M probes may run: of the default tile or of the plane-major order's.
int64_t grad_pass_tiles(const ld_csr* B, int M, int vec_f64, const ld_opts* opt) {
  const Shape sh = grad_shape(B, M, vec_f64, opt);
  return std::max(tiles_of(B, sh), tiles_of(B, plane_shape(sh, opt)));
}

// Pattern analysis, cached per (device, row_ptr, col_idx, rows, nnz).  Every user gets:
//  hash:  the pattern hash at analysis time.  Every call that relies on the analysis hashes the
//         pattern again on the device and compares once its results are back (no extra
//         synchronisation); a pattern rewritten in place at the same addresses is then analysed
//         afresh and the call repeated;
//  dist_hist, plane_rows: how far entries sit from the diagonal (stencil plans, plane-major order).
// The gradient adds (full):
//  sym:   every stored (i, j) has its transposed entry (j, i) stored as well;
//  perm:  (sym) the index of the transposed entry of every entry;
//  rp_t, col_t, src_t: (not sym) the pattern of B^T and, for each of its entries, the entry of B it
//         comes from.
// Only the first call on a pattern synchronises for it.
// Stencil plan of a pattern for staged tiles of `tr` rows (see StencilDesc), with the per-call
// buffers of the padded layout (values, accumulators); `mu` serialises the calls that use them.
struct StencilPlan {
  int tr = 0, K = 0, nofs = 0, nruns = 0;
  int run_base[kStencilRuns] = {}, run_delta[kStencilRuns] = {};
  int64_t ntiles = 0, slots = 0;  // tiles, entry slots (ntiles * tr * K)
  uint16_t* lcol = nullptr;
  int32_t* emap = nullptr;
  int64_t* dslot = nullptr;  // [d] slot of each row's diagonal entry
  void* ent = nullptr;       // packed entries, ent_bytes per slot
  void* hacc = nullptr;      // adjoint accumulators, hacc_bytes per slot
  size_t ent_bytes = 0, hacc_bytes = 0;
  std::mutex mu;             // held by the call that uses ent and hacc (StencilHold)
  // Per-call buffers for a call's value type and vector precision, grown on demand (the caller holds
  // mu, and the previous holder's stream has drained).
  int ensure(size_t eb, size_t hb) {
    if (eb > ent_bytes) {
      if (ent) (void)hipFree(ent);
      ent = nullptr;
      ent_bytes = 0;
      hipError_t e = hipMalloc(&ent, (size_t)std::max<int64_t>(slots, 1) * eb);
      if (e != hipSuccess) {
        ent = nullptr;
        return fail(LD_ENOMEM, "hipMalloc for the stencil plan's entries: %s", hipGetErrorString(e));
      }
      ent_bytes = eb;
    }
    if (hb > hacc_bytes) {
      if (hacc) (void)hipFree(hacc);
      hacc = nullptr;
      hacc_bytes = 0;
      hipError_t e = hipMalloc(&hacc, (size_t)std::max<int64_t>(slots, 1) * hb);
      if (e != hipSuccess) {
        hacc = nullptr;
        return fail(LD_ENOMEM, "hipMalloc for the stencil plan's accumulators: %s", hipGetErrorString(e));
      }
      hacc_bytes = hb;
    }
    return LD_OK;
  }
  ~StencilPlan() {
    for (void* p : {(void*)lcol, (void*)emap, (void*)dslot, ent, hacc})
      if (p) (void)hipFree(p);
  }
};

struct PatternInfo {
  std::mutex full_mu;
  bool full = false;  // the gradient's part below (sym, perm or the pattern of B^T) is filled in
  bool sym = false;
  std::mutex stencil_mu;
  std::map<std::pair<int, int>, std::shared_ptr<StencilPlan>> stencil;  // (tr, offset capacity) -> plan, or null:
                                                                        // not a stencil pattern for that tile
  uint64_t dist_hist[kDistBins] = {};  // entries per bit length of |i - j| (launch_distance_hist)
  int64_t plane_rows = 0;  // lattice reach: the pattern's largest |i - j| when (nearly) every entry sits
                           // near the diagonal or near that distance (launch_plane_fit), else 0
  int64_t* perm = nullptr;
  int64_t* rp_t = nullptr;
  int32_t* col_t = nullptr;
  int64_t* src_t = nullptr;
  uint64_t hash = 0;
  uint64_t last_use = 0;
  ~PatternInfo() {
    for (void* p : {(void*)perm, (void*)rp_t, (void*)col_t, (void*)src_t})
      if (p) (void)hipFree(p);
  }
};

struct PatternKey {
  int dev;
  const void *rp, *col;
  int64_t rows, nnz;
  bool operator<(const PatternKey& o) const {
    return std::tie(dev, rp, col, rows, nnz) < std::tie(o.dev, o.rp, o.col, o.rows, o.nnz);
  }
};
std::mutex g_pat_mu;
std::map<PatternKey, std::shared_ptr<PatternInfo>> g_pat;  // entries in use are also held by their call
uint64_t g_pat_clock = 0;
constexpr size_t kPatternCacheEntries = 8;
constexpr int kRetryPattern = 1 << 20;  // internal status: repeat the call with a fresh analysis

int pattern_key(const ld_csr* B, PatternKey& k) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  k = PatternKey{dev, B->row_ptr, B->col_idx, B->rows, B->nnz};
  return LD_OK;
}

// Device allocation owned by a PatternInfo or by a temporary below.
template <typename T>
int dev_alloc(T** p, size_t count, const char* what) {
  *p = nullptr;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(LD_ENOMEM, "hipMalloc for %s: %s", what, hipGetErrorString(e));
  }
  return LD_OK;
}

struct DevTmp {
  void* p = nullptr;
  ~DevTmp() {
    if (p) (void)hipFree(p);
  }
};

// The part of the analysis every user of the cache needs: the pattern hash, the row-distance
// histogram and the lattice reach.
int analyze_light(const ld_csr* B, hipStream_t s, PatternInfo& P) {
  const int64_t d = B->rows, nnz = B->nnz;
  DevTmp scratch;  // [8]: hash (uint64), [64]: distance histogram, [448]: plane fit
  LD_HIP(hipMalloc(&scratch.p, 512));
  uint64_t* hash = reinterpret_cast<uint64_t*>(static_cast<char*>(scratch.p) + 8);
  unsigned long long* hist = reinterpret_cast<unsigned long long*>(static_cast<char*>(scratch.p) + 64);
  unsigned long long* fit = reinterpret_cast<unsigned long long*>(static_cast<char*>(scratch.p) + 448);
  static_assert(64 + kDistBins * 8 <= 448, "pattern analysis scratch");
  LD_HIP(launch_fill_zero(scratch.p, 512, s));
  LD_HIP(launch_pattern_hash(B->row_ptr, B->col_idx, d, nnz, hash, s));
  LD_HIP(launch_distance_hist(B->row_ptr, B->col_idx, d, nnz, hist, s));
  LD_HIP(launch_plane_fit(B->row_ptr, B->col_idx, d, 0, fit, s));
  unsigned long long fit_h[2] = {0, 0};
  LD_HIP(hipMemcpyAsync(&P.hash, hash, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  LD_HIP(hipMemcpyAsync(P.dist_hist, hist, sizeof(P.dist_hist), hipMemcpyDeviceToHost, s));
  LD_HIP(hipMemcpyAsync(fit_h, fit, sizeof(fit_h), hipMemcpyDeviceToHost, s));
  LD_HIP(hipStreamSynchronize(s));
  const int64_t reach = (int64_t)fit_h[0];
  if (reach >= 16) {  // how many entries sit away from both the diagonal and the reach
    LD_HIP(launch_plane_fit(B->row_ptr, B->col_idx, d, reach, fit, s));
    LD_HIP(hipMemcpyAsync(fit_h, fit, sizeof(fit_h), hipMemcpyDeviceToHost, s));
    LD_HIP(hipStreamSynchronize(s));
    if (fit_h[1] * 100 <= (uint64_t)nnz) P.plane_rows = reach;
  }
  return LD_OK;
}

// The gradient's part: whether every entry has its transpose (then the transposed-entry index),
// else the pattern of B^T.
int analyze_full(const ld_csr* B, hipStream_t s, PatternInfo& P) {
  const int64_t d = B->rows, nnz = B->nnz;
  DevTmp flag;
  LD_HIP(hipMalloc(&flag.p, 256));
  int* missing = static_cast<int*>(flag.p);
  int rc = dev_alloc(&P.perm, (size_t)nnz, "the transposed-entry index");
  if (rc) return rc;
  LD_HIP(launch_fill_zero(flag.p, 256, s));
  LD_HIP(launch_transpose_index(B->row_ptr, B->col_idx, d, nnz, P.perm, missing, s));
  int miss = 0;
  LD_HIP(hipMemcpyAsync(&miss, missing, sizeof(int), hipMemcpyDeviceToHost, s));
  LD_HIP(hipStreamSynchronize(s));
  P.sym = miss == 0;
  if (P.sym) return LD_OK;
  (void)hipFree(P.perm);
  P.perm = nullptr;
  if ((rc = dev_alloc(&P.rp_t, (size_t)d + 1, "the pattern of B^T")) || (rc = dev_alloc(&P.col_t, (size_t)nnz, "B^T")) ||
      (rc = dev_alloc(&P.src_t, (size_t)nnz, "B^T")))
    return rc;
  DevTmp cursor, scan;
  LD_HIP(hipMalloc(&cursor.p, (size_t)std::max<int64_t>(d, 1) * 8));
  LD_HIP(hipMalloc(&scan.p, transpose_scratch_bytes(d)));
  LD_HIP(launch_transpose(B->row_ptr, B->col_idx, nullptr, valt_of(B->dtype), d, nnz, P.rp_t, P.col_t, nullptr,
                          static_cast<int64_t*>(cursor.p), scan.p, transpose_scratch_bytes(d), s, P.src_t));
  LD_HIP(hipStreamSynchronize(s));
  return LD_OK;
}

// Completes the gradient's part of an analysis once.
int ensure_full(const ld_csr* B, hipStream_t s, PatternInfo& P) {
  std::lock_guard<std::mutex> lk(P.full_mu);
  if (P.full) return LD_OK;
  const int rc = analyze_full(B, s, P);
  if (rc) return rc;
  P.full = true;
  return LD_OK;
}

// The cached analysis of B's pattern, made on first sight (full: with the gradient's part).
int get_pattern(const ld_csr* B, hipStream_t s, std::shared_ptr<PatternInfo>& out, bool full = true) {
  PatternKey key;
  int rc = pattern_key(B, key);
  if (rc) return rc;
  {
    std::unique_lock<std::mutex> lk(g_pat_mu);
    auto it = g_pat.find(key);
    if (it != g_pat.end()) {
      it->second->last_use = ++g_pat_clock;
      out = it->second;
      lk.unlock();
      return full ? ensure_full(B, s, *out) : LD_OK;
    }
  }
  auto P = std::make_shared<PatternInfo>();
  rc = analyze_light(B, s, *P);
  if (!rc && full) rc = ensure_full(B, s, *P);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_pat_mu);
  if (g_pat.size() >= kPatternCacheEntries) {
    auto lru = g_pat.begin();
    for (auto it = g_pat.begin(); it != g_pat.end(); ++it)
      if (it->second->last_use < lru->second->last_use) lru = it;
    g_pat.erase(lru);
  }
  P->last_use = ++g_pat_clock;
  g_pat[key] = P;
  out = P;
  return LD_OK;
}

void drop_pattern(const ld_csr* B) {
  PatternKey key;
  if (pattern_key(B, key)) return;
  std::lock_guard<std::mutex> lk(g_pat_mu);
  g_pat.erase(key);
}

// Builds the stencil plan on the host from a copy of the pattern, or leaves `out` null when the
// pattern is not one for tiles of `tr` rows: more than `cap` distinct offsets (column - tile's first
// row) outside the tile over all tiles, or more than kStencilRuns runs of them, rows longer than
// kStencilK, a row without its diagonal, or a padded layout more than 1.5 times the stored entries.
// Tiles are independent, so ranges of them are scanned on several host threads.
int build_stencil_plan(const ld_csr* B, hipStream_t s, int tr, int cap, std::shared_ptr<StencilPlan>& out) {
  out.reset();
  const int64_t d = B->rows, nnz = B->nnz;
  if (d <= 0 || nnz <= 0 || nnz > (int64_t)INT32_MAX) return LD_OK;
  std::vector<int64_t> rp((size_t)d + 1);
  std::vector<int32_t> col((size_t)nnz);
  LD_HIP(hipMemcpyAsync(rp.data(), B->row_ptr, (size_t)(d + 1) * 8, hipMemcpyDeviceToHost, s));
  LD_HIP(hipMemcpyAsync(col.data(), B->col_idx, (size_t)nnz * 4, hipMemcpyDeviceToHost, s));
  LD_HIP(hipStreamSynchronize(s));
  int K = 0;
  for (int64_t r = 0; r < d; ++r) K = std::max<int64_t>(K, rp[(size_t)r + 1] - rp[(size_t)r]);
  const int64_t nt = (d + tr - 1) / tr;
  if (K < 1 || K > kStencilK) return LD_OK;
  if (K != 5 && K != 7) K = kStencilK;  // the kernel's padded widths
  std::vector<int64_t> ds((size_t)d, -1);
  if ((double)nt * tr * K > 1.5 * (double)nnz) return LD_OK;
  // distinct outside offsets, per thread, then merged
  const int nthr = (int)std::max<int64_t>(1, std::min<int64_t>({16, (int64_t)std::thread::hardware_concurrency(),
                                                                 (nt + 4095) / 4096}));
  std::vector<std::vector<int64_t>> offs((size_t)nthr);
  std::vector<char> over((size_t)nthr, 0);
  auto scan = [&](int w) {
    const int64_t t0 = nt * w / nthr, t1 = nt * (w + 1) / nthr;
    std::vector<int64_t>& o = offs[(size_t)w];
    for (int64_t t = t0; t < t1 && !over[(size_t)w]; ++t) {
      const int64_t r0 = t * tr, r1 = std::min<int64_t>(d, r0 + tr);
      for (int64_t e = rp[(size_t)r0]; e < rp[(size_t)r1]; ++e) {
        const int64_t c = col[(size_t)e];
        if (c < r0 || c >= r1) o.push_back(c - r0);
      }
      if ((t & 63) == 63 || t + 1 == t1) {
        std::sort(o.begin(), o.end());
        o.erase(std::unique(o.begin(), o.end()), o.end());
        if ((int64_t)o.size() > cap) over[(size_t)w] = 1;
      }
    }
  };
  {
    std::vector<std::thread> th;
    for (int w = 1; w < nthr; ++w) th.emplace_back(scan, w);
    scan(0);
    for (auto& x : th) x.join();
  }
  std::vector<int64_t> ofs;
  for (int w = 0; w < nthr; ++w) {
    if (over[(size_t)w]) return LD_OK;
    ofs.insert(ofs.end(), offs[(size_t)w].begin(), offs[(size_t)w].end());
  }
  std::sort(ofs.begin(), ofs.end());
  ofs.erase(std::unique(ofs.begin(), ofs.end()), ofs.end());
  if ((int64_t)ofs.size() > cap) return LD_OK;
  // the list as runs of consecutive offsets, passed to the kernel by value
  std::vector<std::pair<int64_t, int64_t>> runs;
  for (int64_t o : ofs) {
    if (!runs.empty() && runs.back().first + runs.back().second == o)
      ++runs.back().second;
    else
      runs.push_back({o, 1});
  }
  if ((int)runs.size() > kStencilRuns) return LD_OK;
  // a halo beyond three tiles' worth of rows (3-D lattices: four) stages more than the entries save,
  // and the staged kernels load at most three halo rows per thread (on the 128^3 GMRF five halo
  // rows per thread gave the staged adjoint 0.372 ms against 0.387 ms explicit but the staged step
  // 0.243 against 0.234 ms, and slowed the 2-D grids' staged kernels by 3 %)
  if ((int64_t)ofs.size() > 3 * (int64_t)tr) return LD_OK;
  for (auto& r : runs)
    if (r.first < INT32_MIN / 2 || r.first > INT32_MAX / 2) return LD_OK;
  // padded layout: slot (t * tr + lr) * K + k
  const int64_t slots = nt * tr * K;
  std::vector<uint16_t> lc((size_t)slots, 0);
  std::vector<int32_t> em((size_t)slots, -1);
  auto fill = [&](int w) {
    const int64_t t0 = nt * w / nthr, t1 = nt * (w + 1) / nthr;
    for (int64_t t = t0; t < t1; ++t) {
      const int64_t r0 = t * tr, r1 = std::min<int64_t>(d, r0 + tr);
      for (int64_t r = r0; r < r1; ++r) {
        int64_t k = 0;
        for (int64_t e = rp[(size_t)r]; e < rp[(size_t)r + 1]; ++e, ++k) {
          const int64_t c = col[(size_t)e];
          const size_t slot = (size_t)(r * K + k);
          em[slot] = (int32_t)e;
          if (c == r) ds[(size_t)r] = (int64_t)slot;
          lc[slot] = (c >= r0 && c < r1)
                         ? (uint16_t)(c - r0)
                         : (uint16_t)(tr + (std::lower_bound(ofs.begin(), ofs.end(), c - r0) - ofs.begin()));
        }
      }
    }
  };
  {
    std::vector<std::thread> th;
    for (int w = 1; w < nthr; ++w) th.emplace_back(fill, w);
    fill(0);
    for (auto& x : th) x.join();
  }
  for (int64_t r = 0; r < d; ++r)
    if (ds[(size_t)r] < 0) return LD_OK;  // the shift's derivative is read off the diagonal entries
  auto P = std::make_shared<StencilPlan>();
  P->tr = tr;
  P->K = K;
  P->nofs = (int)ofs.size();
  P->nruns = (int)runs.size();
  int base = 0;
  for (int i = 0; i < P->nruns; ++i) {
    P->run_base[i] = base;
    P->run_delta[i] = (int)runs[(size_t)i].first - base;  // halo index j of run i has offset j + delta
    base += (int)runs[(size_t)i].second;
  }
  P->ntiles = nt;
  P->slots = slots;
  int rc;
  if ((rc = dev_alloc(&P->lcol, (size_t)slots, "the stencil plan")) || (rc = dev_alloc(&P->emap, (size_t)slots, "the stencil plan")) ||
      (rc = dev_alloc(&P->dslot, (size_t)d, "the stencil plan")))
    return rc;
  LD_HIP(hipMemcpyAsync(P->dslot, ds.data(), (size_t)d * 8, hipMemcpyHostToDevice, s));
  LD_HIP(hipMemcpyAsync(P->lcol, lc.data(), (size_t)slots * 2, hipMemcpyHostToDevice, s));
  LD_HIP(hipMemcpyAsync(P->emap, em.data(), (size_t)slots * 4, hipMemcpyHostToDevice, s));
  LD_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
  out = P;
  return LD_OK;
}

// Staged tiles only pay on patterns whose entries stay near their rows; a pattern is taken for a
// stencil plan only when at most 1 % of its entries reach farther from their row than a 4 MiB window
// of vector rows (one XCD's L2), which keeps scattered patterns from a pointless host scan.
constexpr size_t kLocalWindowBytes = 4u << 20;

bool local_pattern(const PatternInfo& P, int64_t nnz, size_t row_bytes) {
  const uint64_t window = kLocalWindowBytes / std::max<size_t>(row_bytes, 1);
  uint64_t far = 0;
  for (int b = 1; b < kDistBins; ++b)  // bin b holds distances in [2^(b-1), 2^b - 1]
    if (((1ull << b) - 1) > window) far += P.dist_hist[b];
  return far * 100 <= (uint64_t)std::max<int64_t>(nnz, 0);
}

// Plane-major tile order.  On a lattice in its natural order (3-D: neighbours at +-1, +-N, +-N^2)
// row order re-reads a gathered vector row about 2 N^2 rows after its first use; once that span
// of each vector outgrows an XCD's L2 the far neighbours are fetched twice.  Visiting the tiles
// plane by plane within a column of each plane per XCD keeps three planes of a column in L2.
// Taken for passes whose vector rows over one plane reach kPlaneMinBytes, when the tile height
// divides the plane into a multiple of 8 tiles and the tiles fill whole planes (LD_PLANE=0 keeps
// row order; LD_PLANE=1 drops the size condition, for tests).
constexpr double kPlaneMinBytes = 1u << 20;

int plane_tiles(const PatternInfo* P, const Shape& sh, int64_t d, size_t row_bytes) {
  const char* e = std::getenv("LD_PLANE");
  if (e && e[0] == '0') return 0;
  const bool any_size = e && e[0] == '1';
  if (!P || P->plane_rows <= 0 || sh.tile_rows <= 0 || d <= 0) return 0;
  const int64_t reach = P->plane_rows;
  if (!any_size && (double)reach * (double)row_bytes < kPlaneMinBytes) return 0;
  if (reach % sh.tile_rows) return 0;
  const int64_t per = reach / sh.tile_rows;
  const int64_t nt = (d + sh.tile_rows - 1) / sh.tile_rows;
  if (per % 8 || nt % per || per > INT32_MAX) return 0;
  return (int)per;
}

// The stencil plans whose per-call buffers a gradient call uses, locked in the order its passes
// need them (every call takes its full-size passes' plan before its last pass's), and released
// only once the call's stream has drained.
struct StencilHold {
  hipStream_t s = nullptr;
  std::vector<StencilPlan*> held;
  std::vector<std::unique_lock<std::mutex>> locks;
  void take(StencilPlan* p) {
    if (std::find(held.begin(), held.end(), p) != held.end()) return;
    held.push_back(p);
    locks.emplace_back(p->mu);
  }
  ~StencilHold() {
    if (!locks.empty()) (void)hipStreamSynchronize(s);
  }
};

// LD_STENCIL=0 keeps the shifted adjoint on global gathers (for tests).
bool stencil_enabled() {
  const char* e = std::getenv("LD_STENCIL");
  return !(e && e[0] == '0');
}

// Staged tile of a gradient pass's shape: rows and offset capacity (0 rows: no staged form).
std::pair<int, int> stencil_shape(const Shape& sh, size_t vb) {
  const int tr = stencil_tile_rows(sh.lpr_log2);
  if (tr > kStencilRows) return {0, 0};
  const size_t slot_bytes = 2 * (size_t)((1 << sh.lpr_log2) * sh.vpl) * vb;
  const int slots = (int)(kStencilLdsBytes / slot_bytes);
  if (slots <= tr) return {0, 0};
  return {tr, slots - tr};
}

// The cached stencil plan of a pattern for a pass shape (built on first use); null when the pattern
// is not a stencil pattern for that tile.
int get_stencil(PatternInfo& P, const ld_csr* B, hipStream_t s, const Shape& sh, size_t vb,
                std::shared_ptr<StencilPlan>& out) {
  out.reset();
  const std::pair<int, int> ss = stencil_shape(sh, vb);
  if (ss.first == 0 || B->rows <= 0) return LD_OK;
  std::lock_guard<std::mutex> lk(P.stencil_mu);
  auto it = P.stencil.find(ss);
  if (it != P.stencil.end()) {
    out = it->second;
    return LD_OK;
  }
  std::shared_ptr<StencilPlan> S;
  const int rc = build_stencil_plan(B, s, ss.first, ss.second, S);
  if (rc) return rc;
  P.stencil[ss] = S;
  out = S;
  return LD_OK;
}

// Staged steps of an estimator call (ld_logdet_cheb, ld_logdet_taylor) on a stencil pattern: the
// cached plan of the pattern (only the cheap part of its analysis), its packed entries refreshed
// from the values of this call and held until the call's stream has drained, and the pattern hashed
// again during the call.  A pattern rewritten in place since the plan was made is caught by check()
// once the stream has drained: the caller analyses it again and repeats the call.
struct StagedSteps {
  std::shared_ptr<PatternInfo> pat;
  std::shared_ptr<StencilPlan> sp;
  StencilHold hold;
  StencilDesc sd{};
  uint64_t* hash_dev = nullptr;  // 256 bytes of the caller's workspace
  uint64_t hash = 0;
  int steps = 0;

  // Sets the plan up when B is a stencil pattern for the shape sh (one probe tile); sh then takes
  // the staged tile height (a power-of-two number of stencil tiles) and ntiles follows it.
  int setup(const ld_csr* B, hipStream_t s, Shape& sh, int64_t& ntiles, int M, size_t vb, int valt, int vec_f64,
            const ld_opts* opt, void* hash_buf) {
    hold.s = s;
    hash_dev = static_cast<uint64_t*>(hash_buf);
    const int64_t d = B->rows;
    if (!stencil_enabled() || d <= 0 || vec_f64 || valt == VAL_F64 || sh.probe_tiles != 1) return LD_OK;
    int rc = get_pattern(B, s, pat, false);
    if (rc) return rc;
    if (local_pattern(*pat, B->nnz, (size_t)M * vb)) {
      rc = get_stencil(*pat, B, s, sh, vb, sp);
      if (rc) return rc;
    }
    if (!sp) return LD_OK;
    // on the 4096^2 grid 256-row blocks run the staged step in 1.33 ms, the 320-row default in 1.42 ms
    sh = plane_shape(sh, opt);
    ntiles = (d + sh.tile_rows - 1) / sh.tile_rows;
    hold.take(sp.get());
    rc = sp->ensure(stencil_entry_bytes(valt), 0);
    if (rc) return rc;
    sd.ent = sp->ent;
    sd.hacc = sp->hacc;
    sd.K = sp->K;
    sd.nofs = sp->nofs;
    sd.nruns = sp->nruns;
    std::copy(sp->run_base, sp->run_base + kStencilRuns, sd.run_base);
    std::copy(sp->run_delta, sp->run_delta + kStencilRuns, sd.run_delta);
    LD_HIP(launch_stencil_pack(B->values, valt, sp->emap, sp->lcol, sp->slots, sp->ent, s));
    LD_HIP(launch_pattern_hash(B->row_ptr, B->col_idx, d, B->nnz, hash_dev, s));
    return LD_OK;
  }
  // Whether a step of this form would run on the staged tiles.
  bool staged_for(const StepLaunch& L, int vec_f64, int valt, int gsrc, int dsrc, int psrc, int mu) const {
    return sp && step_stencil_supported(L, vec_f64, valt, gsrc, dsrc, psrc, mu);
  }
  // One step, staged when the plan and the step's form allow it.
  hipError_t step(const StepLaunch& L, int vec_f64, int valt, int gsrc, int dsrc, int psrc, int mu, hipStream_t s) {
    if (staged_for(L, vec_f64, valt, gsrc, dsrc, psrc, mu)) {
      ++steps;
      return launch_step_stencil(L, sd, valt, gsrc, psrc, mu, s);
    }
    return launch_step(L, vec_f64, valt, gsrc, dsrc, psrc, mu, s);
  }
  // Before the call's final synchronisation.
  int enqueue_hash(hipStream_t s) {
    if (sp) LD_HIP(hipMemcpyAsync(&hash, hash_dev, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    return LD_OK;
  }
  // After it: the pattern is the one the plan was made for, or kRetryPattern / an error.
  int check(const ld_csr* B, bool allow_retry) {
    if (!sp || hash == pat->hash) return LD_OK;
    drop_pattern(B);
    if (!allow_retry) return fail(LD_EINVAL, "the pattern of B changed while the estimate ran");
    return kRetryPattern;
  }
};

// Shared body of ld_logdet_cheb and ld_logabsdet_cheb.
// fixed_plan: no autotuning and no timing events (the planner's default shape), for callers that
// must not allocate; the workspace is then always opt->workspace.
// staged: the product-identity steps may run on staged stencil tiles (ld_logdet_cheb); the pattern
// is then hashed again during the call, and a pattern found rewritten in place returns kRetryPattern
// (allow_retry) or an error.
int run_forward(const ld_csr* B, const ld_csr* Ct_in, bool ns, double a, double b, int n, int M_out, uint64_t seed,
                const ld_opts* opt, hipStream_t s, ld_result* out, bool fixed_plan = false, bool staged = false,
                bool allow_retry = true) {
  const int valt = valt_of(B->dtype);
  const int vec_f64 = vec_f64_of(opt, valt);
  const int64_t d = B->rows;
  const int M = padded_probes(M_out, vec_f64, opt);  // probes run; the estimate uses the first M_out
  const bool pair = use_pairs(opt);
  const int nsteps = steps_for(n, pair);
  const int nrows = partial_rows(n, pair);
  const size_t need = fwd_workspace(B, n, M_out, vec_f64, ns, opt);
  Workspace ws;
  int rc = get_workspace(opt, need, s, ws);
  if (rc) return rc;

  FwdPlan p = plan_fwd(B, vec_f64, M, opt);
  Carve cv;
  cv.base = static_cast<char*>(ws.ptr);
  const size_t vecb = (size_t)d * M * p.vb;
  void* bufA = cv.take(vecb);
  void* bufB = cv.take(vecb);
  void* bufT = nullptr;
  ld_csr Ct{};
  if (ns) {
    bufT = cv.take(vecb);
    int64_t* rpt = static_cast<int64_t*>(cv.take((size_t)(d + 1) * 8));
    int32_t* colt = static_cast<int32_t*>(cv.take((size_t)B->nnz * 4));
    void* valt_ = cv.take((size_t)B->nnz * val_bytes(valt));
    int64_t* cursor = static_cast<int64_t*>(cv.take((size_t)d * 8));
    void* scan = cv.take(transpose_scratch_bytes(d));
    if (Ct_in) {
      Ct = *Ct_in;
    } else {
      LD_HIP(launch_transpose(B->row_ptr, B->col_idx, B->values, valt, d, B->nnz, rpt, colt, valt_, cursor, scan,
                              transpose_scratch_bytes(d), s));
      Ct = *B;
      Ct.row_ptr = rpt;
      Ct.col_idx = colt;
      Ct.values = valt_;
    }
  }
  const bool tune = !fixed_plan && (!opt || opt->tile == 0) && autotune_enabled() && d >= 65536;
  double* part_base =
      static_cast<double*>(cv.take((size_t)std::max(nrows, 1) * max_tiles(B, vec_f64, M, opt) * M * 8));
  double* red_out = static_cast<double*>(cv.take((size_t)M * std::max(nrows, 1) * 8));
  double* red_tmp = static_cast<double*>(cv.take(reduce_scratch_bytes(nrows, M)));
  const int mu_mode = pair ? MU_PAIR : MU_PROBE;

  // Staged steps on stencil patterns: every step reads W_k's rows (or the probe signs) from LDS tiles.
  StagedSteps st;
  void* hash_buf = cv.take(256);
  if (staged && !ns && !fixed_plan) {
    rc = st.setup(B, s, p.sh, p.ntiles, M, p.vb, valt, vec_f64, opt, hash_buf);
    if (rc) return rc;
  }

  if (tune && !ns && !st.sp) {
    TuneKey key{vec_f64, valt, M, (opt ? opt->probe_tile : 0) * 4 + mu_mode, d, B->nnz};
    Shape sh{};
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune.find(key);
      if (it != g_tune.end()) sh = it->second;
    }
    if (!sh.tile_rows) {
      const std::vector<Shape> shapes = (opt && opt->probe_tile > 0) ? std::vector<Shape>{p.sh}
                                                                      : shape_candidates(vec_f64, M);
      sh = autotune(B, shapes, vec_f64, valt, M, mu_mode, bufA, bufB, part_base, s);
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune[key] = sh;
    }
    if (sh.tile_rows > 0) {
      p.sh = sh;
      p.ntiles = (d + sh.tile_rows - 1) / sh.tile_rows;
    }
  }

  const std::vector<double> c = cheb_coeffs(a, b, n);
  const double alpha = 4.0 / (b - a);
  const double beta = -2.0 * (a + b) / (b - a);
  const double shift = ns ? 0.0 : B->diag_shift;
  const double beff = beta + alpha * shift;
  const int64_t kstride = p.ntiles * M;

  StepTimer tm;
  tm.on = !fixed_plan && opt && opt->timing;
  tm.s = s;

  StepLaunch L{};
  L.nmat = 1;
  L.ntiles = p.ntiles;
  L.tile_rows = p.sh.tile_rows;
  L.M = M;
  L.shape = p.sh;

  auto base_desc = [&](const ld_csr* X) {
    StepDesc D{};
    D.row_ptr = X->row_ptr;
    D.col = X->col_idx;
    D.val = X->values;
    D.seed = seed;
    D.d = d;
    D.active = 1;
    return D;
  };
  // step k writes partial row k (plain) or rows 2k, 2k+1 (pairs)
  auto set_parts = [&](StepDesc& D, int k) {
    D.mu_part = part_base + (int64_t)(pair ? 2 * k : k) * kstride;
    D.mu_part2 = pair ? part_base + (int64_t)(2 * k + 1) * kstride : nullptr;
  };

  // W_k lives in: k = 0 -> probe hash, odd k -> A, even k >= 2 -> B.
  auto wbuf = [&](int k) -> void* { return k == 0 ? nullptr : ((k & 1) ? bufA : bufB); };
  LD_HIP(tm.mark(T_OTHER));
  for (int k = 0; k < nsteps && d > 0; ++k) {
    const int gsrc = k == 0 ? SRC_HASH : SRC_BUF;
    const int psrc = k == 0 ? SRC_NONE : (k == 1 ? SRC_HASH : SRC_BUF);
    const double h = k == 0 ? 0.5 : 1.0;  // W_1 = At V carries half of 2 At
    if (!ns) {
      StepDesc D = base_desc(B);
      D.G = wbuf(k);
      D.P = k >= 2 ? wbuf(k - 1) : nullptr;
      D.out = wbuf(k + 1);
      D.ag = h * alpha;
      D.bd = h * beff;
      D.cp = k == 0 ? 0.0 : -1.0;
      set_parts(D, k);
      L.d0 = D;
      LD_HIP(st.step(L, vec_f64, valt, gsrc, SRC_SAME, psrc, mu_mode, s));
      LD_HIP(tm.mark(T_STEP));
    } else {
      // T = C W_k
      StepDesc D1 = base_desc(B);
      D1.G = wbuf(k);
      D1.out = bufT;
      D1.ag = 1.0;
      L.d0 = D1;
      LD_HIP(launch_step(L, vec_f64, valt, gsrc, SRC_NONE, SRC_NONE, MU_NONE, s));
      LD_HIP(tm.mark(T_STEP));
      // W_{k+1} = alpha C^T T + beta W_k - W_{k-1}   (halved at k = 0)
      StepDesc D2 = base_desc(&Ct);
      D2.G = bufT;
      D2.D = wbuf(k);
      D2.P = k >= 2 ? wbuf(k - 1) : nullptr;
      D2.out = wbuf(k + 1);
      D2.ag = h * alpha;
      D2.bd = h * beta;
      D2.cp = k == 0 ? 0.0 : -1.0;
      set_parts(D2, k);
      L.d0 = D2;
      LD_HIP(launch_step(L, vec_f64, valt, SRC_BUF, k == 0 ? SRC_HASH : SRC_BUF, psrc, mu_mode, s));
      LD_HIP(tm.mark(T_STEP));
    }
  }
  std::vector<double> red((size_t)M * std::max(nrows, 1), 0.0);
  if (nrows >= 1 && d > 0) {
    LD_HIP(launch_reduce_moments(part_base, p.ntiles, M, 0, nrows - 1, kstride, red_out, nrows, red_tmp, s));
    LD_HIP(hipMemcpyAsync(red.data(), red_out, (size_t)M * nrows * 8, hipMemcpyDeviceToHost, s));
  }
  rc = st.enqueue_hash(s);
  if (rc) return rc;
  LD_HIP(hipStreamSynchronize(s));
  rc = st.check(B, allow_retry);
  if (rc) return rc;
  std::vector<double> mu((size_t)M_out * (n + 1), 0.0);
  assemble_moments(red, nrows, pair, n, M_out, d, mu);  // rows of red are per probe: the first M_out
  combine(mu, c, n, M_out, d, ns ? 0.5 : 1.0, out, opt);
  out->poly_bound = lemma_bound(a, b, n, d) * (ns ? 0.5 : 1.0);
  out->grad_shift = 0.0;
  out->staged_steps = st.steps;
  tm.report(out);
  return out->flags ? LD_WBOUNDS : LD_OK;
}

int run_taylor(const ld_csr* B, double a, double b, int n, int M, uint64_t seed, const ld_opts* opt, hipStream_t s,
               ld_result* out, bool allow_retry = true) {
  const int valt = valt_of(B->dtype);
  const int vec_f64 = vec_f64_of(opt, valt);
  const int64_t d = B->rows;
  Workspace ws;
  int rc = get_workspace(opt, taylor_workspace(B, n, M, vec_f64, opt), s, ws);
  if (rc) return rc;
  FwdPlan p = plan_fwd(B, vec_f64, M, opt);
  Carve cv;
  cv.base = static_cast<char*>(ws.ptr);
  const size_t vecb = (size_t)d * M * p.vb;
  void* buf[2] = {cv.take(vecb), cv.take(vecb)};
  const int rows = std::max(n, 1);
  double* part_base = static_cast<double*>(cv.take((size_t)rows * max_tiles(B, vec_f64, M, opt) * M * 8));
  double* red_out = static_cast<double*>(cv.take((size_t)M * rows * 8));
  double* red_tmp = static_cast<double*>(cv.take(reduce_scratch_bytes(rows, M)));
  StagedSteps st;
  rc = st.setup(B, s, p.sh, p.ntiles, M, p.vb, valt, vec_f64, opt, cv.take(256));
  if (rc) return rc;
  const int64_t kstride = p.ntiles * M;
  const double scale = a + b;  // B/(a + b) has spectrum in [delta, 1 - delta] (Section 3.1)

  StepTimer tm;
  tm.on = opt && opt->timing;
  tm.s = s;
  StepLaunch L{};
  L.nmat = 1;
  L.ntiles = p.ntiles;
  L.tile_rows = p.sh.tile_rows;
  L.M = M;
  L.shape = p.sh;
  LD_HIP(tm.mark(T_OTHER));
  for (int k = 0; k < n && d > 0; ++k) {  // W_{k+1} = A W_k with W_0 = V from the probe hash
    StepDesc D{};
    D.row_ptr = B->row_ptr;
    D.col = B->col_idx;
    D.val = B->values;
    D.seed = seed;
    D.d = d;
    D.active = 1;
    D.G = k == 0 ? nullptr : buf[(k - 1) & 1];
    D.out = buf[k & 1];
    D.ag = -1.0 / scale;
    D.bd = 1.0 - B->diag_shift / scale;
    D.cp = 0.0;  // no third operand: the general kernel takes the probe hash for it, scaled away
    D.mu_part = part_base + (int64_t)k * kstride;
    L.d0 = D;
    const int gsrc = k == 0 ? SRC_HASH : SRC_BUF;
    const bool bare = k == 0 || st.staged_for(L, vec_f64, valt, gsrc, SRC_SAME, SRC_NONE, MU_PROBE);
    LD_HIP(st.step(L, vec_f64, valt, gsrc, SRC_SAME, bare ? SRC_NONE : SRC_HASH, MU_PROBE, s));
    LD_HIP(tm.mark(T_STEP));
  }
  std::vector<double> red((size_t)M * rows, 0.0);
  if (n >= 1 && d > 0) {
    LD_HIP(launch_reduce_moments(part_base, p.ntiles, M, 0, n - 1, kstride, red_out, n, red_tmp, s));
    LD_HIP(hipMemcpyAsync(red.data(), red_out, (size_t)M * n * 8, hipMemcpyDeviceToHost, s));
  }
  rc = st.enqueue_hash(s);
  if (rc) return rc;
  LD_HIP(hipStreamSynchronize(s));
  rc = st.check(B, allow_retry);
  if (rc) return rc;
  // log det B = d log(a + b) - sum_k tr(A^k)/k: coefficients log(a + b) on mu_0 = v^T v = d and -1/k
  std::vector<double> mu((size_t)M * (n + 1), 0.0), c(n + 1);
  c[0] = std::log(scale);
  for (int k = 1; k <= n; ++k) c[k] = -1.0 / k;
  for (int j = 0; j < M; ++j) {
    mu[(size_t)j * (n + 1)] = (double)d;
    for (int k = 1; k <= n; ++k) mu[(size_t)j * (n + 1) + k] = red[(size_t)j * rows + (k - 1)];
  }
  combine(mu, c, n, M, d, 1.0, out, opt);
  // truncation: |sum_{k>n} tr(A^k)/k| <= d q^{n+1} / ((n+1)(1-q)), q = 1 - delta = b/(a+b)
  const double q = b / scale;
  out->poly_bound = (double)d * std::pow(q, n + 1) / ((n + 1) * (1.0 - q));
  out->grad_shift = 0.0;
  out->staged_steps = st.steps;
  tm.report(out);
  return out->flags ? LD_WBOUNDS : LD_OK;
}

// Diagonal partials any adjoint launch of a gradient call may write: one per tile of the pass
// shapes, and at least the 256 of the staged steps' diagonal sum.
int64_t grad_diag_tiles(const ld_csr* B, int M, int vec_f64, const ld_opts* opt) {
  const GradChunks ch = grad_chunks(M, vec_f64);
  int64_t nt = 0;
  for (int mp : {ch.size, ch.last}) nt = std::max(nt, grad_pass_tiles(B, mp, vec_f64, opt));
  return std::max<int64_t>(nt, 256);  // the staged steps' diagonal sum writes 256 partials
}

size_t grad_workspace_for(const ld_csr* B, int n, int M, int vec_f64, const ld_opts* opt, int stride, bool pair) {
  const size_t vb = vec_f64 ? 8 : 4;
  const GradPlan g = plan_grad(n, pair, stride);
  const GradChunks ch = grad_chunks(M, vec_f64);
  const int64_t nt_full = grad_pass_tiles(B, ch.size, vec_f64, opt);
  const int64_t nt_last = grad_pass_tiles(B, ch.last, vec_f64, opt);
  const int64_t ntiles = grad_diag_tiles(B, M, vec_f64, opt);
  const int64_t part_cols = std::max(nt_full * ch.size, nt_last * ch.last);  // per partial row
  const int rows = std::max(partial_rows(n, g.pair), 1);
  Carve c;
  const size_t vecb = (size_t)B->rows * ch.size * vb;
  for (int i = 0; i < g.nslots + g.nseg_buf + 2; ++i) c.take(vecb);
  c.take((size_t)B->nnz * vb);                       // gradient accumulators
  if (!pair) c.take((size_t)B->nnz * val_bytes(valt_of(B->dtype)));  // values of B^T (adjoint of the plain form)
  c.take(256);                                       // pattern hash
  c.take((size_t)std::max<int64_t>(ntiles, 1) * 8);  // diagonal partials
  c.take(8);                                         // diagonal total
  c.take((size_t)rows * part_cols * 8);              // per-tile moment partials
  c.take((size_t)ch.size * rows * 8);                // reduced partials
  c.take(reduce_scratch_bytes(rows, ch.size));
  return align_up(c.off);
}

// A non-symmetric pattern falls back to the plain recurrence, so size for both plans.
// Checkpoint stride of each form of the gradient (the paired form with the product identities,
// and the plain recurrence that patterns without their transpose run): the caller's, else 1
// (every W_k kept, no recomputation) when that form's plan fits the memory available -- the
// caller's workspace, or half of the device's free memory -- else 0 (ceil(sqrt(steps))).  The
// form is known only once the pattern has been checked, so each is planned on its own: the
// plain form keeps twice as many blocks and may have to recompute where the paired one need not.
struct GradStrides {
  int pair, plain;
};

GradStrides choose_strides(const ld_csr* B, int n, int M, int vec_f64, const ld_opts* opt) {
  if (opt && opt->ckpt_stride > 0) return {opt->ckpt_stride, opt->ckpt_stride};
  size_t avail = 0;
  if (opt && opt->workspace) {
    avail = opt->workspace_bytes;
  } else {
    // counting the library's idle pooled buffers as free: they are reused before anything new is
    // allocated, so a repeated call plans as the first one did
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess) avail = (fr + pool_idle_bytes()) / 2;
  }
  GradStrides st;
  st.pair = grad_workspace_for(B, n, M, vec_f64, opt, 1, true) <= avail ? 1 : 0;
  st.plain = grad_workspace_for(B, n, M, vec_f64, opt, 1, false) <= avail ? 1 : 0;
  return st;
}

// Workspace for either form with its stride.
size_t grad_workspace_strides(const ld_csr* B, int n, int M, int vec_f64, const ld_opts* opt, const GradStrides& st) {
  size_t w = grad_workspace_for(B, n, M, vec_f64, opt, st.plain, false);
  if (use_pairs(opt)) w = std::max(w, grad_workspace_for(B, n, M, vec_f64, opt, st.pair, true));
  return w;
}

size_t grad_workspace(const ld_csr* B, int n, int M, int vec_f64, const ld_opts* opt) {
  return grad_workspace_strides(B, n, M, vec_f64, opt, choose_strides(B, n, M, vec_f64, opt));
}

}  // namespace

// ======================================================================================
// batched
// ======================================================================================

namespace {

// One captured graph for one batch signature, with the device memory it refers to.
struct BatchEntry {
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  void* mem = nullptr;
  double* mu_dev = nullptr;
  int kmax = 0;  // partial rows of the longest member
  bool pair = true;
  uint64_t last_use = 0;
  std::vector<std::vector<double>> coeffs;
  ~BatchEntry() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (mem) (void)hipFree(mem);
  }
};
std::mutex g_batch_mu;
std::map<std::vector<double>, std::unique_ptr<BatchEntry>> g_batch;
uint64_t g_batch_clock = 0;               // use counter for least-recently-used eviction
constexpr size_t kBatchCacheEntries = 8;  // captured graphs (with their device memory) kept

double bits_of(const void* p) {
  uint64_t u = (uint64_t)(uintptr_t)p;
  double x;
  std::memcpy(&x, &u, 8);
  return x;
}

int build_batch(int count, const ld_csr* Bs, const double* a, const double* b, const int* n, int M, uint64_t seed,
                int vec_f64, int valt, bool pair, const Shape& sh, BatchEntry& E) {
  const size_t vb = vec_f64 ? 8 : 4;
  // kmax: steps of the longest member; rmax: partial rows of the longest member
  int kmax = 0, rmax = 0;
  std::vector<int> rows_i(count);
  for (int i = 0; i < count; ++i) {
    kmax = std::max(kmax, steps_for(n[i], pair));
    rows_i[i] = partial_rows(n[i], pair);
    rmax = std::max(rmax, rows_i[i]);
  }
  E.kmax = rmax;
  E.pair = pair;
  // Tiles in order of decreasing step count (stable): the members still active at step k are then
  // a prefix of the tile list, and node k dispatches only that prefix (active_tiles[k]) instead of
  // every member's tiles with the finished ones returning at once.
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return steps_for(n[x], pair) > steps_for(n[y], pair); });
  std::vector<int64_t> tile_begin(count), tile_range(2 * (size_t)count);
  int64_t ntiles = 0;
  for (int i : order) {
    tile_begin[i] = ntiles;
    ntiles += (Bs[i].rows + sh.tile_rows - 1) / sh.tile_rows;
    tile_range[2 * (size_t)i] = tile_begin[i];
    tile_range[2 * (size_t)i + 1] = ntiles;
  }
  std::vector<int64_t> active_tiles(std::max(kmax, 1), 0);
  for (int k = 0; k < kmax; ++k)
    for (int i : order)
      if (steps_for(n[i], pair) > k) active_tiles[k] = tile_range[2 * (size_t)i + 1];
  std::vector<int32_t> tile_mat(ntiles);
  std::vector<int64_t> tile_row0(ntiles);
  for (int i = 0; i < count; ++i)
    for (int64_t t = tile_range[2 * (size_t)i]; t < tile_range[2 * (size_t)i + 1]; ++t) {
      tile_mat[t] = i;
      tile_row0[t] = (t - tile_begin[i]) * sh.tile_rows;
    }
  // device layout
  Carve c;
  std::vector<void*> bufA(count), bufB(count);
  std::vector<size_t> offA(count), offB(count);
  for (int i = 0; i < count; ++i) {
    c.take((size_t)Bs[i].rows * M * vb);
    offA[i] = c.off - (size_t)Bs[i].rows * M * vb;
    c.take((size_t)Bs[i].rows * M * vb);
    offB[i] = c.off - (size_t)Bs[i].rows * M * vb;
  }
  const int64_t kstride = ntiles * M;
  c.take((size_t)std::max(rmax, 1) * kstride * 8);
  const size_t off_part = c.off - (size_t)std::max(rmax, 1) * kstride * 8;
  c.take((size_t)count * M * (rmax + 1) * 8);
  const size_t off_mu = c.off - (size_t)count * M * (rmax + 1) * 8;
  c.take((size_t)std::max(kmax, 1) * count * sizeof(StepDesc));
  const size_t off_desc = c.off - (size_t)std::max(kmax, 1) * count * sizeof(StepDesc);
  c.take((size_t)ntiles * 4);
  const size_t off_tm = c.off - (size_t)ntiles * 4;
  c.take((size_t)ntiles * 8);
  const size_t off_tr = c.off - (size_t)ntiles * 8;
  c.take((size_t)count * 16);
  const size_t off_tb = c.off - (size_t)count * 16;
  c.take((size_t)count * 4);
  const size_t off_n = c.off - (size_t)count * 4;
  hipError_t e = hipMalloc(&E.mem, align_up(c.off));
  if (e != hipSuccess)
    return fail(LD_ENOMEM, "hipMalloc(%zu) for the batch: %s", align_up(c.off), hipGetErrorString(e));
  char* base = static_cast<char*>(E.mem);
  for (int i = 0; i < count; ++i) {
    bufA[i] = base + offA[i];
    bufB[i] = base + offB[i];
  }
  double* part = reinterpret_cast<double*>(base + off_part);
  E.mu_dev = reinterpret_cast<double*>(base + off_mu);
  StepDesc* descs = reinterpret_cast<StepDesc*>(base + off_desc);
  int32_t* d_tm = reinterpret_cast<int32_t*>(base + off_tm);
  int64_t* d_tr = reinterpret_cast<int64_t*>(base + off_tr);
  int64_t* d_tb = reinterpret_cast<int64_t*>(base + off_tb);
  int* d_n = reinterpret_cast<int*>(base + off_n);

  std::vector<StepDesc> hd((size_t)std::max(kmax, 1) * count);
  E.coeffs.resize(count);
  for (int i = 0; i < count; ++i) {
    E.coeffs[i] = cheb_coeffs(a[i], b[i], n[i]);
    const double alpha = 4.0 / (b[i] - a[i]);
    const double beta = -2.0 * (a[i] + b[i]) / (b[i] - a[i]);
    const double beff = beta + alpha * Bs[i].diag_shift;
    auto wbuf = [&](int k) -> void* { return k == 0 ? nullptr : ((k & 1) ? bufA[i] : bufB[i]); };
    for (int k = 0; k < kmax; ++k) {
      StepDesc& D = hd[(size_t)k * count + i];
      D = StepDesc{};
      D.row_ptr = Bs[i].row_ptr;
      D.col = Bs[i].col_idx;
      D.val = Bs[i].values;
      D.seed = seed + (uint64_t)i;
      D.d = Bs[i].rows;
      D.active = k < steps_for(n[i], pair) ? 1 : 0;
      const double h = k == 0 ? 0.5 : 1.0;
      D.G = wbuf(k);
      D.P = k >= 2 ? wbuf(k - 1) : nullptr;
      D.out = wbuf(k + 1);
      D.ag = h * alpha;
      D.bd = h * beff;
      D.cp = k == 0 ? 0.0 : -1.0;
      D.mu_part = part + (int64_t)(pair ? 2 * k : k) * kstride + tile_begin[i] * M;
      D.mu_part2 = pair ? part + (int64_t)(2 * k + 1) * kstride + tile_begin[i] * M : nullptr;
      D.tile0 = tile_begin[i];
    }
  }
  LD_HIP(hipMemcpy(descs, hd.data(), hd.size() * sizeof(StepDesc), hipMemcpyHostToDevice));
  LD_HIP(hipMemcpy(d_tm, tile_mat.data(), tile_mat.size() * 4, hipMemcpyHostToDevice));
  LD_HIP(hipMemcpy(d_tr, tile_row0.data(), tile_row0.size() * 8, hipMemcpyHostToDevice));
  LD_HIP(hipMemcpy(d_tb, tile_range.data(), tile_range.size() * 8, hipMemcpyHostToDevice));
  LD_HIP(hipMemcpy(d_n, rows_i.data(), (size_t)count * 4, hipMemcpyHostToDevice));

  if (rmax == 0) return LD_OK;  // every member has degree 0: nothing to run, no graph
  // capture every step and the reduction on a private stream
  hipStream_t cs;
  LD_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  for (int k = 0; k < kmax && err == hipSuccess; ++k) {
    StepLaunch L{};
    L.descs = descs + (size_t)k * count;
    L.nmat = count;
    L.tile_mat = d_tm;
    L.tile_row0 = d_tr;
    L.ntiles = active_tiles[k];
    L.tile_rows = sh.tile_rows;
    L.M = M;
    L.shape = sh;
    if (L.ntiles == 0) continue;
    const int gsrc = k == 0 ? SRC_HASH : SRC_BUF;
    const int psrc = k == 0 ? SRC_NONE : (k == 1 ? SRC_HASH : SRC_BUF);
    err = launch_step(L, vec_f64, valt, gsrc, SRC_SAME, psrc, pair ? MU_PAIR : MU_PROBE, cs);
  }
  if (err == hipSuccess) err = launch_reduce_batched(part, d_tb, d_n, count, M, rmax, kstride, E.mu_dev, cs);
  hipError_t e2 = hipStreamEndCapture(cs, &E.graph);
  (void)hipStreamDestroy(cs);
  if (err != hipSuccess) return fail_hip(err, "batched step capture");
  if (e2 != hipSuccess) return fail_hip(e2, "hipStreamEndCapture");
  LD_HIP(hipGraphInstantiate(&E.exec, E.graph, nullptr, nullptr, 0));
  return LD_OK;
}

}  // namespace

// ======================================================================================
// C ABI
// ======================================================================================

// ------------------------------------------------------------------------------------
// Forward without allocation: the workspace is a fixed device array of the library
// ------------------------------------------------------------------------------------

namespace {

// Device memory of ld_logdet_cheb_noalloc: one copy per GPU the library runs on, held until the
// process ends.  In host code `scratch` names a host-side stand-in, never the device array:
// every host use goes through the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[LD_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;  // device -> device address of its copy of `scratch`

// Address of the current device's `scratch`, looked up once per device (with it current).
int scratch_address(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) {
    *ptr = it->second;
    return LD_OK;
  }
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
  if (!p || reinterpret_cast<uintptr_t>(p) % kAlign) return fail(LD_EHIP, "scratch has no aligned device address");
  g_scratch_addr[dev] = p;
  *ptr = p;
  return LD_OK;
}

}  // namespace

extern "C" {

const char* ld_last_error(void) { return g_err; }

const char* ld_version(void) { return "logdet_cheb 1.0 (gfx950)"; }

static size_t workspace_bytes_impl(const ld_csr* B, int n, int M, int mode, int vec_f64) {
  if (!B || n < 0 || M < 1) return 0;
  const int valt = valt_of(B->dtype);
  ld_opts o{};
  o.vec_f64 = vec_f64 ? 1 : 2;
  const int v64 = vec_f64_of(&o, valt);
  if (mode == 2) return grad_workspace(B, n, M, v64, nullptr);
  if (mode == 3) return taylor_workspace(B, n, M, v64, nullptr);
  return fwd_workspace(B, n, M, v64, mode == 1, nullptr);
}

static int logdet_cheb_impl(const ld_csr* B, double a, double b, int n, int M, uint64_t seed, const ld_opts* opt,
                            void* stream, ld_result* out) {
  int rc = check_csr(B, "B");
  if (rc) return rc;
  rc = check_common(a, b, n, M);
  if (rc) return rc;
  if (!out) return fail(LD_EINVAL, "out is NULL");
  ld_result r{};
  const hipStream_t s = static_cast<hipStream_t>(stream);
  rc = run_forward(B, nullptr, false, a, b, n, M, seed, opt, s, &r, false, true, true);
  if (rc == kRetryPattern) rc = run_forward(B, nullptr, false, a, b, n, M, seed, opt, s, &r, false, true, false);
  if (rc < 0) return rc;
  *out = r;
  return rc;
}

static int logdet_cheb_noalloc_impl(const ld_csr* B, double a, double b, int n, int M, uint64_t seed,
                                    const ld_opts* opt, void* stream, ld_result* out) {
  int rc = check_csr(B, "B");
  if (rc) return rc;
  rc = check_common(a, b, n, M);
  if (rc) return rc;
  if (!out) return fail(LD_EINVAL, "out is NULL");
  if (opt && opt->workspace) return fail(LD_EINVAL, "ld_logdet_cheb_noalloc takes no workspace (opt->workspace)");
  ld_opts o{};
  if (opt) o = *opt;
  const int vec_f64 = vec_f64_of(&o, valt_of(B->dtype));
  const size_t need = fwd_workspace(B, n, M, vec_f64, false, &o);
  if (need > (size_t)LD_NOALLOC_SCRATCH_BYTES)
    return fail(LD_EWORKSPACE, "ld_logdet_cheb_noalloc needs %zu bytes of scratch; its limit is %zu bytes", need,
                (size_t)LD_NOALLOC_SCRATCH_BYTES);
  void* base = nullptr;
  rc = scratch_address(&base);
  if (rc) return rc;
  o.workspace = base;
  o.workspace_bytes = LD_NOALLOC_SCRATCH_BYTES;
  ld_result r{};
  rc = run_forward(B, nullptr, false, a, b, n, M, seed, &o, static_cast<hipStream_t>(stream), &r, true);
  if (rc < 0) return rc;
  *out = r;
  return rc;
}

static int logdet_taylor_impl(const ld_csr* B, double a, double b, int n, int M, uint64_t seed, const ld_opts* opt,
                              void* stream, ld_result* out) {
  int rc = check_csr(B, "B");
  if (rc) return rc;
  rc = check_common(a, b, n, M);
  if (rc) return rc;
  if (!out) return fail(LD_EINVAL, "out is NULL");
  ld_result r{};
  const hipStream_t s = static_cast<hipStream_t>(stream);
  rc = run_taylor(B, a, b, n, M, seed, opt, s, &r, true);
  if (rc == kRetryPattern) rc = run_taylor(B, a, b, n, M, seed, opt, s, &r, false);
  if (rc < 0) return rc;
  *out = r;
  return rc;
}

static int logabsdet_cheb_impl(const ld_csr* C, const ld_csr* Ct, double smin, double smax, int n, int M, uint64_t seed,
                               const ld_opts* opt, void* stream, ld_result* out) {
  int rc = check_csr(C, "C");
  if (rc) return rc;
  if (Ct) {
    rc = check_csr(Ct, "Ct");
    if (rc) return rc;
    if (Ct->rows != C->rows || Ct->nnz != C->nnz || Ct->dtype != C->dtype)
      return fail(LD_EINVAL, "Ct does not match C in size, nnz or dtype");
  }
  if (C->diag_shift != 0.0) return fail(LD_EINVAL, "C->diag_shift must be 0 for Algorithm 2");
  if (!std::isfinite(smin) || !std::isfinite(smax) || !(smin > 0.0) || !(smax > smin))
    return fail(LD_EINVAL, "singular-value bounds must satisfy 0 < smin < smax; got %g, %g", smin, smax);
  rc = check_common(smin * smin, smax * smax, n, M);
  if (rc) return rc;
  if (!out) return fail(LD_EINVAL, "out is NULL");
  ld_result r{};
  rc = run_forward(C, Ct, true, smin * smin, smax * smax, n, M, seed, opt, static_cast<hipStream_t>(stream), &r);
  if (rc < 0) return rc;
  *out = r;
  return rc;
}

static int laplacian_minor_impl(const ld_csr* adj, int64_t hub, int64_t* row_ptr_out, int32_t* col_out, void* val_out,
                                int32_t val_dtype, int64_t* max_degree, void* stream) {
  int rc = check_csr(adj, "adj");
  if (rc) return rc;
  if (adj->rows < 2) return fail(LD_EINVAL, "a graph needs at least 2 vertices; got %lld", (long long)adj->rows);
  if (hub < 0 || hub >= adj->rows) return fail(LD_EINVAL, "hub %lld outside [0, %lld)", (long long)hub,
                                               (long long)adj->rows);
  if (val_dtype != LD_F64 && val_dtype != LD_F32) return fail(LD_EDTYPE, "minor values must be LD_F64 or LD_F32");
  if (!row_ptr_out || !col_out || !val_out || !max_degree) return fail(LD_EINVAL, "an output pointer is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int64_t hb[2];
  LD_HIP(hipMemcpyAsync(hb, adj->row_ptr + hub, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  LD_HIP(hipStreamSynchronize(s));
  const int64_t deg_hub = hb[1] - hb[0];
  if (deg_hub != adj->rows - 1)
    return fail(LD_EINVAL, "vertex %lld has degree %lld, not %lld: it is not adjacent to every other vertex",
                (long long)hub, (long long)deg_hub, (long long)(adj->rows - 1));
  const int64_t m = adj->rows - 1;
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (m + 255) / 256));
  Workspace ws;
  rc = get_workspace(nullptr, (size_t)nb * 16, s, ws);
  if (rc) return rc;
  int64_t* mx_part = static_cast<int64_t*>(ws.ptr);
  int64_t* bad_part = mx_part + nb;
  LD_HIP(launch_laplacian_minor(adj->row_ptr, adj->col_idx, adj->rows, hub, deg_hub, row_ptr_out, col_out, val_out,
                                val_dtype == LD_F64 ? VAL_F64 : VAL_F32, mx_part, bad_part, nb, s));
  std::vector<int64_t> h(2 * (size_t)nb);
  LD_HIP(hipMemcpyAsync(h.data(), mx_part, h.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  LD_HIP(hipStreamSynchronize(s));
  int64_t mx = 0, bad = 0;
  for (int i = 0; i < nb; ++i) {
    mx = std::max(mx, h[i]);
    bad += h[nb + i];
  }
  if (bad)
    return fail(LD_EINVAL, "%lld vertices miss the hub, carry a self loop or repeat a neighbour", (long long)bad);
  *max_degree = mx;
  return LD_OK;
}

static int log_spanning_trees_impl(const ld_csr* adj, int64_t hub, int n, int M, uint64_t seed, int method,
                                   const ld_opts* opt, void* stream, ld_result* out) {
  if (method != 0 && method != 1) return fail(LD_EINVAL, "method must be 0 (Algorithm 1) or 1 (Algorithm 2)");
  if (!out) return fail(LD_EINVAL, "out is NULL");
  int rc = check_csr(adj, "adj");
  if (rc) return rc;
  rc = check_common(1.0, 2.0, n, M);
  if (rc) return rc;
  if (adj->rows < 2) return fail(LD_EINVAL, "a graph needs at least 2 vertices; got %lld", (long long)adj->rows);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t m = adj->rows - 1;
  const int64_t nnz_out = adj->nnz - m;  // valid once the hub's degree is checked to be m
  if (nnz_out < m) return fail(LD_EINVAL, "adjacency has too few entries for a hub of degree %lld", (long long)m);
  const bool f64 = opt && opt->vec_f64 == 1;
  Carve c;
  c.take((size_t)(m + 1) * 8);
  c.take((size_t)nnz_out * 4);
  c.take((size_t)nnz_out * (f64 ? 8 : 4));
  Workspace ws;
  rc = get_workspace(nullptr, align_up(c.off), s, ws);
  if (rc) return rc;
  c = Carve{static_cast<char*>(ws.ptr)};
  int64_t* rp = static_cast<int64_t*>(c.take((size_t)(m + 1) * 8));
  int32_t* col = static_cast<int32_t*>(c.take((size_t)nnz_out * 4));
  void* val = c.take((size_t)nnz_out * (f64 ? 8 : 4));
  int64_t dmax = 0;
  rc = ld_laplacian_minor(adj, hub, rp, col, val, f64 ? LD_F64 : LD_F32, &dmax, stream);
  if (rc) return rc;
  ld_result r{};
  r.n = n;
  r.M = M;
  if (dmax <= 1) {  // every other vertex hangs off the hub alone: L(hub) = I and the tree is unique
    if (opt && opt->probe_out)
      for (int j = 0; j < M; ++j) opt->probe_out[j] = 0.0;
    *out = r;
    return LD_OK;
  }
  ld_csr L{m, m, nnz_out, rp, col, val, f64 ? LD_F64 : LD_F32, 0, 0.0};
  const double hi = 2.0 * (double)dmax - 1.0;  // spectrum of L(hub) lies in [1, 2 Delta_max - 1]
  if (method == 0)
    rc = run_forward(&L, nullptr, false, 1.0, hi, n, M, seed, opt, s, &r);
  else
    rc = run_forward(&L, &L, true, 1.0, hi * hi, n, M, seed, opt, s, &r);  // C = L(hub) is its own transpose
  if (rc < 0) return rc;
  *out = r;
  return rc;
}

// Rows per work item of the batched Gershgorin pass.
constexpr int64_t kGershRows = 4096;

static int gershgorin_batched_impl(int count, const ld_csr* Bs, double* a, double* b, void* stream) {
  if (count < 1 || !Bs || !a || !b) return fail(LD_EINVAL, "invalid batch arguments");
  for (int i = 0; i < count; ++i) {
    char name[32];
    snprintf(name, sizeof(name), "Bs[%d]", i);
    int rc = check_csr(&Bs[i], name);
    if (rc) return rc;
    if (Bs[i].rows < 1) return fail(LD_EINVAL, "Bs[%d] is empty: no spectrum", i);
    if (Bs[i].dtype != Bs[0].dtype) return fail(LD_EDTYPE, "all batch matrices must share one dtype");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<GershItem> items;
  std::vector<int> owner;
  for (int i = 0; i < count; ++i)
    for (int64_t r = 0; r < Bs[i].rows; r += kGershRows) {
      items.push_back(GershItem{Bs[i].row_ptr, Bs[i].col_idx, Bs[i].values, Bs[i].diag_shift, r,
                                std::min(Bs[i].rows, r + kGershRows)});
      owner.push_back(i);
    }
  const int ni = (int)items.size();
  Carve c;
  c.take(sizeof(GershItem) * ni);
  c.take((size_t)ni * 16);
  Workspace ws;
  int rc = get_workspace(nullptr, align_up(c.off), s, ws);
  if (rc) return rc;
  Carve cv;
  cv.base = static_cast<char*>(ws.ptr);
  GershItem* d_items = static_cast<GershItem*>(cv.take(sizeof(GershItem) * ni));
  double* part = static_cast<double*>(cv.take((size_t)ni * 16));
  LD_HIP(hipMemcpyAsync(d_items, items.data(), sizeof(GershItem) * ni, hipMemcpyHostToDevice, s));
  LD_HIP(launch_gershgorin_batched(d_items, ni, valt_of(Bs[0].dtype), part, part + ni, s));
  std::vector<double> h(2 * (size_t)ni);
  LD_HIP(hipMemcpyAsync(h.data(), part, h.size() * 8, hipMemcpyDeviceToHost, s));
  LD_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < count; ++i) {
    a[i] = INFINITY;
    b[i] = -INFINITY;
  }
  for (int k = 0; k < ni; ++k) {
    a[owner[k]] = std::min(a[owner[k]], h[k]);
    b[owner[k]] = std::max(b[owner[k]], h[ni + k]);
  }
  return LD_OK;
}

static int gershgorin_impl(const ld_csr* B, double* a, double* b, void* stream) {
  int rc = check_csr(B, "B");
  if (rc) return rc;
  if (!a || !b) return fail(LD_EINVAL, "a or b is NULL");
  if (B->rows == 0) return fail(LD_EINVAL, "empty matrix has no spectrum");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nb = (int)std::min<int64_t>(1024, (B->rows + 255) / 256);
  Workspace ws;
  rc = get_workspace(nullptr, (size_t)nb * 16, s, ws);
  if (rc) return rc;
  double* lo = static_cast<double*>(ws.ptr);
  double* hi = lo + nb;
  LD_HIP(launch_gershgorin(B->row_ptr, B->col_idx, B->values, valt_of(B->dtype), B->diag_shift, B->rows, lo, hi, nb,
                           s));
  std::vector<double> h(2 * (size_t)nb);
  LD_HIP(hipMemcpyAsync(h.data(), lo, h.size() * 8, hipMemcpyDeviceToHost, s));
  LD_HIP(hipStreamSynchronize(s));
  double l = INFINITY, u = -INFINITY;
  for (int i = 0; i < nb; ++i) {
    l = std::min(l, h[i]);
    u = std::max(u, h[nb + i]);
  }
  *a = l;
  *b = u;
  return LD_OK;
}

static int probes_impl(uint64_t seed, int M, int64_t rows, int8_t* out, void* stream) {
  if (M < 1 || rows < 0 || (!out && rows > 0)) return fail(LD_EINVAL, "invalid probe block arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  LD_HIP(launch_probes(seed, M, rows, out, s));
  LD_HIP(hipStreamSynchronize(s));
  return LD_OK;
}

static int transpose_impl(const ld_csr* C, int64_t* row_ptr_t, int32_t* col_t, void* val_t, void* stream) {
  int rc = check_csr(C, "C");
  if (rc) return rc;
  if (!row_ptr_t || (C->nnz > 0 && (!col_t || !val_t))) return fail(LD_EINVAL, "NULL output buffer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace ws;
  rc = get_workspace(nullptr, align_up((size_t)C->rows * 8) + transpose_scratch_bytes(C->rows), s, ws);
  if (rc) return rc;
  int64_t* cursor = static_cast<int64_t*>(ws.ptr);
  void* scan = static_cast<char*>(ws.ptr) + align_up((size_t)C->rows * 8);
  LD_HIP(launch_transpose(C->row_ptr, C->col_idx, C->values, valt_of(C->dtype), C->rows, C->nnz, row_ptr_t, col_t,
                          val_t, cursor, scan, transpose_scratch_bytes(C->rows), s));
  LD_HIP(hipStreamSynchronize(s));
  return LD_OK;
}

static int copy_impl(void* dst, const void* src, size_t bytes, void* stream, double* ms) {
  if ((!dst || !src) && bytes) return fail(LD_EINVAL, "NULL pointer");
  if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15u)
    return fail(LD_EINVAL, "ld_copy needs 16-byte aligned pointers");
  hipStream_t s = static_cast<hipStream_t>(stream);
  struct Events {
    hipEvent_t e[2] = {nullptr, nullptr};
    ~Events() {
      for (auto x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } ev;
  LD_HIP(hipEventCreate(&ev.e[0]));
  LD_HIP(hipEventCreate(&ev.e[1]));
  LD_HIP(hipEventRecord(ev.e[0], s));
  LD_HIP(launch_copy(dst, src, bytes, s));
  LD_HIP(hipEventRecord(ev.e[1], s));
  LD_HIP(hipEventSynchronize(ev.e[1]));
  float t = 0.f;
  LD_HIP(hipEventElapsedTime(&t, ev.e[0], ev.e[1]));
  if (ms) *ms = t;
  return LD_OK;
}

// The gradient's forms (the pattern's analysis is cached, see PatternInfo):
//  * paired (default, symmetric pattern): ceil(n/2) products with the product identities, which take
//    B = B^T as Algorithm 1 does; the single-gather adjoint runs on B and each stored entry gets the
//    derivative along symmetric perturbations (G_ij + G_ji) / 2;
//  * plain (a pattern without its transpose, or opt->plain_recurrence): Algorithm 1's recurrence as
//    written, n products, and the adjoint y_k = c_k v + 2 At^T y_{k+1} - y_{k+2} on B^T: the
//    single-gather kernel on B^T applies B^T in its product and accumulates, at B^T's entry (j, i),
//    the derivative with respect to B's entry (i, j), which an index map then carries back.  No
//    symmetry is assumed: each stored entry gets dGamma/dB_ij on its own.
static int grad_body(const ld_csr* B, double a, double b, int n, int M, uint64_t seed, double grad_output,
                     void* grad_values, int grad_dtype, const ld_opts* opt, void* stream, ld_result* out,
                     bool allow_retry) {
  int rc = check_csr(B, "B");
  if (rc) return rc;
  rc = check_common(a, b, n, M);
  if (rc) return rc;
  if (!out) return fail(LD_EINVAL, "out is NULL");
  if (grad_dtype != LD_F64 && grad_dtype != LD_F32) return fail(LD_EDTYPE, "grad_dtype must be LD_F64 or LD_F32");
  if (!grad_values && B->nnz > 0) return fail(LD_EINVAL, "grad_values is NULL");
  if (!std::isfinite(grad_output)) return fail(LD_EINVAL, "grad_output is not finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int valt = valt_of(B->dtype);
  const int vec_f64 = vec_f64_of(opt, valt);
  const int64_t d = B->rows;
  const size_t vb = vec_f64 ? 8 : 4;
  // the probes run in passes of ch.size (the last one ch.last); the gradient accumulators and
  // the per-probe moments collect over the passes
  const GradChunks ch = grad_chunks(M, vec_f64);
  const int64_t nt_max = grad_diag_tiles(B, M, vec_f64, opt);
  const int64_t part_cols = std::max(grad_pass_tiles(B, ch.size, vec_f64, opt) * ch.size,
                                     grad_pass_tiles(B, ch.last, vec_f64, opt) * ch.last);
  const GradStrides strides = choose_strides(B, n, M, vec_f64, opt);
  const size_t need = grad_workspace_strides(B, n, M, vec_f64, opt, strides);
  std::shared_ptr<PatternInfo> pat;
  if (d > 0) {
    rc = get_pattern(B, s, pat);
    if (rc) return rc;
  }
  const bool sym_pattern = !pat || pat->sym;
  const bool pair_form = use_pairs(opt) && sym_pattern;
  Workspace ws;
  rc = get_workspace(opt, need, s, ws);
  if (rc) return rc;
  Carve cv;
  cv.base = static_cast<char*>(ws.ptr);
  const GradPlan g = plan_grad(n, pair_form, pair_form ? strides.pair : strides.plain);
  const bool pair = g.pair;
  const int nrows = partial_rows(n, pair);
  const size_t vecb = (size_t)d * ch.size * vb;
  std::vector<void*> slots(g.nslots), seg(g.nseg_buf);
  for (auto& p : slots) p = cv.take(vecb);
  for (auto& p : seg) p = cv.take(vecb);
  void* Ya = cv.take(vecb);
  void* Yb = cv.take(vecb);
  void* Gacc = cv.take((size_t)B->nnz * vb);
  // the adjoint's matrix: B itself (paired form), or B^T (plain form)
  void* val_t = pair ? nullptr : cv.take((size_t)B->nnz * val_bytes(valt));
  uint64_t* hash_dev = static_cast<uint64_t*>(cv.take(256));
  if (d > 0) LD_HIP(launch_pattern_hash(B->row_ptr, B->col_idx, d, B->nnz, hash_dev, s));
  const int64_t* adj_rp = B->row_ptr;
  const int32_t* adj_col = B->col_idx;
  const void* adj_val = B->values;
  if (!pair && B->nnz > 0) {
    const int64_t* src = sym_pattern ? pat->perm : pat->src_t;  // B^T's entry u is B's entry src[u]
    LD_HIP(launch_gather_values(B->values, valt, src, B->nnz, val_t, s));
    if (!sym_pattern) {
      adj_rp = pat->rp_t;
      adj_col = pat->col_t;
    }
    adj_val = val_t;
  }
  double* gdiag_part = static_cast<double*>(cv.take((size_t)std::max<int64_t>(nt_max, 1) * 8));
  double* gdiag_tot = static_cast<double*>(cv.take(8));
  const int rows_alloc = std::max(nrows, 1);
  double* part = static_cast<double*>(cv.take((size_t)rows_alloc * part_cols * 8));
  double* red_out = static_cast<double*>(cv.take((size_t)ch.size * rows_alloc * 8));
  double* red_tmp = static_cast<double*>(cv.take(reduce_scratch_bytes(rows_alloc, ch.size)));

  const std::vector<double> c = cheb_coeffs(a, b, n);
  const double alpha = 4.0 / (b - a);
  const double beta = -2.0 * (a + b) / (b - a);
  const double beff = beta + alpha * B->diag_shift;
  // Seed coefficients with the product identities (see assemble_moments): the estimate is
  // const + sum_k al[k] W_k^T W_{k+1} + sum_k be[k] W_{k+1}^T W_{k+1}, k = 0..m-1.
  std::vector<double> al(g.m + 1, 0.0), be(g.m + 1, 0.0);
  if (pair) {
    for (int k = 0; k < g.m; ++k) {
      if (2 * k + 2 <= n) be[k] = 2.0 * c[2 * k + 2];
      if (k >= 1 && 2 * k + 1 <= n) al[k] = 2.0 * c[2 * k + 1];
    }
    if (n >= 1) {
      al[0] = c[1];
      for (int k = 1; k < g.m; ++k)
        if (2 * k + 1 <= n) al[0] -= c[2 * k + 1];
    }
  }

  StepTimer tm;
  tm.on = opt && opt->timing;
  tm.s = s;
  LD_HIP(launch_fill_zero(Gacc, (size_t)B->nnz * vb, s));
  LD_HIP(launch_fill_zero(gdiag_part, (size_t)std::max<int64_t>(nt_max, 1) * 8, s));
  LD_HIP(tm.mark(T_OTHER));
  // Adjoint form.  Plain: single-gather on B^T.  Paired (symmetric pattern): the shifted two-gather
  // form for local patterns (two vector blocks less per step), otherwise the single-gather form with
  // the explicit seed (LD_GRAD_SYM=0 keeps the two-gather form there, for tests).
  // The shifted form is taken on its own only with staged tiles (its two gathers per entry from
  // global memory are slower than the explicit form's one): when the pattern is a stencil pattern
  // for the passes' tiles.
  const int form = grad_form_override();
  const bool stencil_on = stencil_enabled();
  bool shifted = pair && form == 1;
  if (pair && form < 0 && pat && stencil_on && local_pattern(*pat, B->nnz, (size_t)ch.size * vb)) {
    std::shared_ptr<StencilPlan> sp0;
    rc = get_stencil(*pat, B, s, grad_shape(B, ch.size, vec_f64, opt), vb, sp0);
    if (rc) return rc;
    shifted = sp0 != nullptr;
  }
  const bool sym = !pair || (!shifted && sym_pattern && sym_enabled());
  // Shifted adjoint: Y holds yh_j = y_j + eps_j w_{j-1}, with eps_j = eps_{j+2} + al[j] - al[j-1]
  // (eps_{top+1} = eps_{top+2} = 0), which cancels every w_{j-1} term of the seed, and step j runs
  // its product on z = yh_{j+1} + kap_j w_j, kap_j = al[j] - eps_{j+1} + eps_{j+2}, using
  // w_{j+1} = 2 At w_j - w_{j-1}:  yh_j = 2 At z - yh_{j+2} + 2 be[j-1] w_j,  yh_top = 2 be[top-1] w_top.
  std::vector<double> eps(g.top + 3, 0.0);
  if (shifted)
    for (int j = g.top; j >= 1; --j) eps[j] = eps[j + 2] + (j < (int)al.size() ? al[j] : 0.0) - al[j - 1];
  std::vector<double> red((size_t)M * rows_alloc, 0.0);  // per-probe partial rows, all passes
  StencilHold sp_hold;
  sp_hold.s = s;
  int staged_passes = 0;  // passes whose adjoint ran on staged stencil tiles
  int plane0 = 0;         // the first pass's plane-major order (tiles per plane)
  int staged_steps = 0;   // forward steps on staged stencil tiles, over all passes

  for (int pass = 0; pass < ch.count; ++pass) {
    const int probe0 = pass * ch.size;  // a multiple of 64 whenever there is more than one pass
    const uint64_t pseed = pass_seed(seed, probe0);
    const int Mp = pass + 1 < ch.count ? ch.size : ch.last;
    Shape sh = grad_shape(B, Mp, vec_f64, opt);
    {
      Shape ps = plane_shape(sh, opt);
      ps.plane = plane_tiles(pat.get(), ps, d, (size_t)Mp * vb);
      if (ps.plane) sh = ps;
    }
    std::shared_ptr<StencilPlan> sp;  // staged tiles of this pass's shifted adjoint
    if (shifted && stencil_on && pat) {
      rc = get_stencil(*pat, B, s, sh, vb, sp);
      if (rc) return rc;
    }
    if (sp && !sh.plane) sh = plane_shape(sh, opt);  // the staged step's tile, as in the estimator
    if (pass == 0) plane0 = sh.plane;
    const int64_t ntiles = tiles_of(B, sh);
    const int64_t kstride = ntiles * Mp;
    StencilDesc sd{};
    if (sp) {
      ++staged_passes;
      sp_hold.take(sp.get());  // its per-call buffers, until this call's stream has drained
      rc = sp->ensure(stencil_entry_bytes(valt), vb);
      if (rc) return rc;
      sd = StencilDesc{};
      sd.ent = sp->ent;
      sd.hacc = sp->hacc;
      sd.K = sp->K;
      sd.nofs = sp->nofs;
      sd.nruns = sp->nruns;
      std::copy(sp->run_base, sp->run_base + kStencilRuns, sd.run_base);
      std::copy(sp->run_delta, sp->run_delta + kStencilRuns, sd.run_delta);
      LD_HIP(launch_stencil_pack(B->values, valt, sp->emap, sp->lcol, sp->slots, sp->ent, s));
      LD_HIP(launch_fill_zero(sp->hacc, (size_t)sp->slots * vb, s));
    }
    StepLaunch L{};
    L.nmat = 1;
    L.ntiles = ntiles;
    L.tile_rows = sh.tile_rows;
    L.M = Mp;
    L.shape = sh;
    auto step = [&](int gsrc, int psrc, int mu, const void* G, const void* P, void* o, double h, double cp,
                    int k) -> hipError_t {
      StepDesc D{};
      D.row_ptr = B->row_ptr;
      D.col = B->col_idx;
      D.val = B->values;
      D.seed = pseed;
      D.d = d;
      D.active = 1;
      D.G = G;
      D.P = P;
      D.out = o;
      D.ag = h * alpha;
      D.bd = h * beff;
      D.cp = cp;
      if (mu != MU_NONE) {
        D.mu_part = part + (int64_t)(pair ? 2 * k : k) * kstride;
        D.mu_part2 = pair ? part + (int64_t)(2 * k + 1) * kstride : nullptr;
      }
      L.d0 = D;
      if (sp && step_stencil_supported(L, vec_f64, valt, gsrc, SRC_SAME, psrc, mu)) {
        ++staged_steps;
        return launch_step_stencil(L, sd, valt, gsrc, psrc, mu, s);
      }
      return launch_step(L, vec_f64, valt, gsrc, SRC_SAME, psrc, mu, s);
    };

    // forward recurrence with checkpoints: W_k lives in bufW[k] (nullptr = probe hash)
    std::vector<void*> bufW(g.m + 2, nullptr);
    void* R0 = seg[0];
    void* R1 = seg[1];
    for (int k = 0; k < g.m && d > 0; ++k) {
      void* o;
      if (g.slot_of[k + 1] >= 0) {
        o = slots[g.slot_of[k + 1]];
      } else {
        void* prev = k >= 1 ? bufW[k - 1] : nullptr;
        if (prev == R0 || prev == R1)
          o = prev;
        else
          o = (bufW[k] == R0) ? R1 : R0;
      }
      const int gsrc = k == 0 ? SRC_HASH : SRC_BUF;
      const int psrc = k == 0 ? SRC_NONE : (k == 1 ? SRC_HASH : SRC_BUF);
      LD_HIP(step(gsrc, psrc, pair ? MU_PAIR : MU_PROBE, bufW[k], k >= 2 ? bufW[k - 1] : nullptr, o,
                  k == 0 ? 0.5 : 1.0, k == 0 ? 0.0 : -1.0, k));
      LD_HIP(tm.mark(T_STEP));
      bufW[k + 1] = o;
    }
    if (nrows >= 1 && d > 0) {
      LD_HIP(launch_reduce_moments(part, ntiles, Mp, 0, nrows - 1, kstride, red_out, nrows, red_tmp, s));
      LD_HIP(hipMemcpyAsync(red.data() + (size_t)probe0 * nrows, red_out, (size_t)Mp * nrows * 8,
                            hipMemcpyDeviceToHost, s));
    }

    // backward.  A symmetric pattern lets each row accumulate its transposed entries from the
    // rows of y_{j+1} that the SpMM gathers anyway (one gather per nonzero instead of two).
    auto ckpt = [&](int k) -> void* { return k == 0 ? nullptr : slots[g.slot_of[k]]; };
    if (n >= 1 && d > 0) {
      // y_top: c_n V (plain) or al[top-1] W_{top-1} + 2 be[top-1] W_top (pairs; W_0 = V)
      if (!pair) {
        LD_HIP(launch_seed(Ya, vec_f64, nullptr, nullptr, nullptr, c[n], 0.0, 0.0, 0.0, pseed, d, Mp, s));
      } else if (shifted) {
        const int t = g.top;
        LD_HIP(launch_seed(Ya, vec_f64, ckpt(t), nullptr, nullptr, 0.0, 2.0 * be[t - 1], 0.0, 0.0, pseed, d, Mp, s));
      } else {
        const int t = g.top;
        LD_HIP(launch_seed(Ya, vec_f64, ckpt(t), t - 1 >= 1 ? ckpt(t - 1) : nullptr, nullptr,
                           t - 1 == 0 ? al[t - 1] : 0.0, 2.0 * be[t - 1], al[t - 1], 0.0, pseed, d, Mp, s));
      }
      LD_HIP(tm.mark(T_OTHER));
      void* y1 = Ya;       // y_{j+1}
      void* y2 = nullptr;  // y_{j+2}
      AdjDesc A{};
      A.row_ptr = adj_rp;
      A.col = adj_col;
      A.val = adj_val;
      A.Gacc = Gacc;
      A.gdiag_part = gdiag_part;
      A.seed = pseed;
      A.d = d;
      A.ag = alpha;
      A.bd = beff;
      A.cp = -1.0;
      for (int q = g.nseg - 1; q >= 0; --q) {
        const int lo = g.lo[q], hi = g.hi[q];
        // segW[i] = W_{lo-1+i}, i = 0 .. hi-lo+1 (+1 with pairs: W_{hi+1})
        std::vector<void*> segW(hi - lo + 3, nullptr);
        segW[0] = ckpt(lo - 1);
        segW[1] = ckpt(lo);
        for (int i = 2; i <= hi - lo + 1; ++i) {
          const int k = lo - 1 + i;  // recompute W_k = 2 At W_{k-1} - W_{k-2}
          const bool p_hash = (k - 2) == 0;
          LD_HIP(step(SRC_BUF, p_hash ? SRC_HASH : SRC_BUF, MU_NONE, segW[i - 1], p_hash ? nullptr : segW[i - 2],
                      seg[i - 2], 1.0, -1.0, 0));
          LD_HIP(tm.mark(T_STEP));
          segW[i] = seg[i - 2];
        }
        if (pair) segW[hi - lo + 2] = ckpt(hi + 1);
        for (int j = hi; j >= lo; --j) {
          void* o = y2 ? y2 : (y1 == Ya ? Yb : Ya);
          A.Y1 = y1;
          A.Y2 = y2;
          A.out = o;
          A.W = segW[j - lo + 1];
          A.gw = 2.0;
          A.ck = A.ce = 0.0;
          if (!pair) {
            A.cv = c[j];
            A.cw = A.cwm = A.cwp = 0.0;
            A.Wm = A.Wp = nullptr;
          } else if (shifted) {
            A.cw = 2.0 * be[j - 1];
            A.cv = A.cwm = A.cwp = 0.0;
            A.Wm = A.Wp = nullptr;
            A.ck = al[j] - eps[j + 1] + eps[j + 2];
            A.ce = eps[j + 1];
          } else {
            A.cw = 2.0 * be[j - 1];
            A.cv = j - 1 == 0 ? al[j - 1] : 0.0;  // W_0 = V
            A.Wm = j - 1 == 0 ? nullptr : segW[j - lo];
            A.cwm = al[j - 1];
            A.Wp = segW[j - lo + 2];
            A.cwp = al[j];
          }
          if (sp)
            LD_HIP(launch_adjoint_stencil(A, sd, Mp, sh, vec_f64, valt, y2 != nullptr, false, s));
          else
            LD_HIP(launch_adjoint(A, Mp, sh, vec_f64, valt, true, false, y2 != nullptr, sym, s));
          LD_HIP(tm.mark(T_ADJ));
          y2 = y1;
          y1 = o;
        }
      }
      // the y_1 w_0^T term, w_0 = v: on the staged tiles into their accumulators when the form allows,
      // else by the general kernel into entry order after them
      A.Y1 = y1;
      A.Y2 = nullptr;
      A.out = nullptr;
      A.W = nullptr;
      A.Wm = A.Wp = nullptr;
      A.cv = A.cw = A.cwm = A.cwp = 0.0;
      A.ck = 0.0;
      A.ce = shifted ? eps[1] : 0.0;  // y_1 = yh_1 - eps_1 w_0
      A.gw = 1.0;
      const bool staged_close = sp && adjoint_stencil_sddmm_supported(vec_f64, valt, sh, sd);
      if (staged_close) LD_HIP(launch_adjoint_stencil(A, sd, Mp, sh, vec_f64, valt, false, true, s));
      if (sp) {  // the staged steps' accumulators: the shift's derivative off the diagonal, then entry order
        LD_HIP(launch_stencil_diag_sum(sp->hacc, vec_f64, sp->dslot, d, gdiag_part, s));
        LD_HIP(launch_stencil_unpack(sp->hacc, vec_f64, sp->emap, sp->slots, Gacc, s));
      }
      if (!staged_close) LD_HIP(launch_adjoint(A, Mp, sh, vec_f64, valt, false, true, false, sym, s));
      LD_HIP(tm.mark(T_OTHER));  // an SDDMM without the product: not timed with the adjoint steps
    }
  }
  const double scale = grad_output * (2.0 / (b - a)) / M;
  if (B->nnz > 0) {
    const int of64 = grad_dtype == LD_F64;
    if (pair)  // the derivative along symmetric perturbations, (G_ij + G_ji)/2
      LD_HIP(launch_sym_scale(Gacc, vec_f64, pat->perm, B->nnz, scale, grad_values, of64, s));
    else if (sym_pattern)  // B^T has B's pattern: entry (i, j) reads the accumulator of (j, i)
      LD_HIP(launch_perm_scale(Gacc, vec_f64, pat->perm, B->nnz, scale, grad_values, of64, 0, s));
    else  // B^T's entry u belongs to B's entry src_t[u]
      LD_HIP(launch_perm_scale(Gacc, vec_f64, pat->src_t, B->nnz, scale, grad_values, of64, 1, s));
  }
  double gd = 0.0;
  if (nt_max > 0) {
    LD_HIP(launch_sum_doubles(gdiag_part, nt_max, gdiag_tot, s));
    LD_HIP(hipMemcpyAsync(&gd, gdiag_tot, 8, hipMemcpyDeviceToHost, s));
  }
  uint64_t hash = 0;
  if (d > 0) LD_HIP(hipMemcpyAsync(&hash, hash_dev, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  LD_HIP(tm.mark(T_OTHER));
  LD_HIP(hipStreamSynchronize(s));
  if (pat && hash != pat->hash) {
    // the pattern at these addresses is not the one analysed: the caller analyses it again and
    // repeats the call, once this call's buffers are released
    drop_pattern(B);
    if (!allow_retry) return fail(LD_EINVAL, "the pattern of B changed while the gradient ran");
    return kRetryPattern;
  }
  std::vector<double> mu((size_t)M * (n + 1), 0.0);
  assemble_moments(red, nrows, pair, n, M, d, mu);
  ld_result r{};
  combine(mu, c, n, M, d, 1.0, &r, opt);
  r.poly_bound = lemma_bound(a, b, n, d);
  r.grad_shift = scale * gd;
  r.adjoint_form = !pair      ? LD_ADJ_PLAIN
                   : shifted  ? (staged_passes == ch.count ? LD_ADJ_SHIFTED_STAGED : LD_ADJ_SHIFTED)
                   : sym      ? LD_ADJ_EXPLICIT_SINGLE
                              : LD_ADJ_EXPLICIT_TWO;
  r.plane_tiles = plane0;
  r.staged_steps = staged_steps;
  tm.report(&r);
  *out = r;
  return r.flags ? LD_WBOUNDS : LD_OK;
}

static int logdet_cheb_grad_impl(const ld_csr* B, double a, double b, int n, int M, uint64_t seed, double grad_output,
                                 void* grad_values, int grad_dtype, const ld_opts* opt, void* stream, ld_result* out) {
  const int rc = grad_body(B, a, b, n, M, seed, grad_output, grad_values, grad_dtype, opt, stream, out, true);
  if (rc != kRetryPattern) return rc;
  return grad_body(B, a, b, n, M, seed, grad_output, grad_values, grad_dtype, opt, stream, out, false);
}

static int logdet_cheb_batched_impl(int count, const ld_csr* Bs, const double* a, const double* b, const int* n, int M,
                                    uint64_t seed, const ld_opts* opt, void* stream, ld_result* outs) {
  if (count < 1 || !Bs || !n || !outs || (!a) != (!b)) return fail(LD_EINVAL, "invalid batch arguments");
  if (M < 1 || M > 4096) return fail(LD_EINVAL, "probe count M=%d out of range [1, 4096]", M);
  std::vector<double> ga, gb;
  if (!a) {  // Gershgorin bounds of every member in one pass
    ga.resize(count);
    gb.resize(count);
    int rc = gershgorin_batched_impl(count, Bs, ga.data(), gb.data(), stream);
    if (rc) return rc;
    a = ga.data();
    b = gb.data();
  }
  for (int i = 0; i < count; ++i) {
    char name[32];
    snprintf(name, sizeof(name), "Bs[%d]", i);
    int rc = check_csr(&Bs[i], name);
    if (rc) return rc;
    rc = check_common(a[i], b[i], n[i], M);
    if (rc) return rc;
    if (Bs[i].rows < 1) return fail(LD_EINVAL, "Bs[%d] is empty", i);
    if (Bs[i].dtype != Bs[0].dtype) return fail(LD_EDTYPE, "all batch matrices must share one dtype");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int valt = valt_of(Bs[0].dtype);
  const int vec_f64 = vec_f64_of(opt, valt);
  const int Mr = padded_probes(M, vec_f64, opt);  // probes the graph runs; results use the first M
  Shape sh = base_shape(vec_f64, Mr);
  const int rpi = rows_per_iter(sh);
  int64_t tot_d = 0, tot_nnz = 0;
  for (int i = 0; i < count; ++i) {
    tot_d += Bs[i].rows;
    tot_nnz += Bs[i].nnz;
  }
  // as for one matrix: the LDS slice capacity, lowered until the whole batch spreads over >= 1024 tiles
  const bool fixed_tile = opt && opt->tile > 0;
  const int tile = fixed_tile ? opt->tile : with_tile(sh, tot_d, tot_nnz, 0).tile_rows;
  sh.tile_rows = (tile + rpi - 1) / rpi * rpi;
  const bool tune = !fixed_tile && autotune_enabled() && tot_d >= 65536;

  const bool pair = use_pairs(opt);
  std::vector<double> key = {(double)count, (double)Mr, (double)(seed >> 32), (double)(seed & 0xffffffffu),
                             (double)vec_f64, fixed_tile ? (double)sh.tile_rows : 0.0, pair ? 1.0 : 0.0};
  for (int i = 0; i < count; ++i) {
    const double v[] = {bits_of(Bs[i].row_ptr), bits_of(Bs[i].col_idx), bits_of(Bs[i].values), (double)Bs[i].rows,
                        (double)Bs[i].nnz, (double)Bs[i].dtype, Bs[i].diag_shift, a[i], b[i], (double)n[i]};
    key.insert(key.end(), v, v + 10);
  }
  std::lock_guard<std::mutex> lk(g_batch_mu);
  auto it = g_batch.find(key);
  BatchEntry* E;
  if (it == g_batch.end()) {
    if (g_batch.size() >= kBatchCacheEntries) {  // every graph has finished: each call synchronises
      auto lru = g_batch.begin();
      for (auto jt = g_batch.begin(); jt != g_batch.end(); ++jt)
        if (jt->second->last_use < lru->second->last_use) lru = jt;
      g_batch.erase(lru);
    }
    std::unique_ptr<BatchEntry> ent;
    if (!tune) {
      ent = std::make_unique<BatchEntry>();
      int rc = build_batch(count, Bs, a, b, n, Mr, seed, vec_f64, valt, pair, sh, *ent);
      if (rc) return rc;
    } else {
      // The batch's autotuner: build the graph for each candidate shape (the full probe block at
      // three tile heights, narrower probe tiles at the tallest), time one replay of each after a
      // warm-up replay, keep the fastest.  Runs once per batch signature; later calls replay it.
      std::vector<Shape> cands;
      const std::vector<Shape> shapes = shape_candidates(vec_f64, Mr);
      for (size_t si = 0; si < shapes.size(); ++si) {
        const std::vector<int> tiles = tile_candidates(shapes[si], tot_d, tot_nnz);
        for (size_t ti = 0; ti < tiles.size() && (si == 0 || ti == 0); ++ti) {
          Shape c = shapes[si];
          c.tile_rows = tiles[ti];
          cands.push_back(c);
        }
      }
      float best = INFINITY;
      for (const Shape& c : cands) {
        auto cand = std::make_unique<BatchEntry>();
        int rc = build_batch(count, Bs, a, b, n, Mr, seed, vec_f64, valt, pair, c, *cand);
        if (rc) {
          if (ent) continue;  // keep the best graph built so far (e.g. out of memory for this one)
          return rc;
        }
        float ms = 0.f;
        if (cand->exec) {
          hipEvent_t e0, e1;
          LD_HIP(hipEventCreate(&e0));
          if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return fail(LD_EHIP, "hipEventCreate failed");
          }
          hipError_t he = hipGraphLaunch(cand->exec, s);
          if (he == hipSuccess) he = hipEventRecord(e0, s);
          if (he == hipSuccess) he = hipGraphLaunch(cand->exec, s);
          if (he == hipSuccess) he = hipEventRecord(e1, s);
          if (he == hipSuccess) he = hipEventSynchronize(e1);
          if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
          (void)hipEventDestroy(e0);
          (void)hipEventDestroy(e1);
          if (he != hipSuccess) return fail_hip(he, "batch autotuning replay");
        }
        if (!ent || ms < best) {
          best = ms;
          ent = std::move(cand);
        }
        if (!ent->exec) break;  // nothing to launch (every degree 0): any shape will do
      }
    }
    E = ent.get();
    g_batch[key] = std::move(ent);
  } else {
    E = it->second.get();
  }
  E->last_use = ++g_batch_clock;
  StepTimer tm;
  tm.on = opt && opt->timing;
  tm.s = s;
  LD_HIP(tm.mark(T_OTHER));
  if (E->exec) LD_HIP(hipGraphLaunch(E->exec, s));
  LD_HIP(tm.mark(T_STEP));
  const int kmax = E->kmax;
  std::vector<double> mu_all((size_t)count * Mr * (kmax + 1));
  if (kmax > 0) LD_HIP(hipMemcpyAsync(mu_all.data(), E->mu_dev, mu_all.size() * 8, hipMemcpyDeviceToHost, s));
  LD_HIP(hipStreamSynchronize(s));
  int status = LD_OK;
  for (int i = 0; i < count; ++i) {
    const int rows = partial_rows(n[i], pair);
    std::vector<double> red((size_t)M * std::max(rows, 1), 0.0);
    for (int j = 0; j < M; ++j)
      for (int r = 0; r < rows; ++r) red[(size_t)j * rows + r] = mu_all[((size_t)i * Mr + j) * (kmax + 1) + r + 1];
    std::vector<double> mu((size_t)M * (n[i] + 1));
    assemble_moments(red, rows, pair, n[i], M, Bs[i].rows, mu);
    ld_result r{};
    combine(mu, E->coeffs[i], n[i], M, Bs[i].rows, 1.0, &r, nullptr);
    r.poly_bound = lemma_bound(a[i], b[i], n[i], Bs[i].rows);
    tm.report(&r);
    if (tm.on) r.kernel_launches = kmax;
    outs[i] = r;
    if (r.flags) status = LD_WBOUNDS;
  }
  return status;
}

// Number of eigenvalues below x of the symmetric tridiagonal matrix with diagonal a and
// squared off-diagonals b2 (b2[0] unused), by the Sturm sequence of its LDL^T pivots.
static int sturm_below(const std::vector<double>& a, const std::vector<double>& b2, double x) {
  int cnt = 0;
  double q = a[0] - x;
  for (size_t i = 0; i < a.size(); ++i) {
    if (i > 0) q = a[i] - x - b2[i] / (q != 0.0 ? q : 1e-300);
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// The idx-th smallest eigenvalue (0-based) of that tridiagonal, by bisection.
static double tridiag_eig(const std::vector<double>& a, const std::vector<double>& b2, int idx) {
  double lo = INFINITY, hi = -INFINITY;
  const size_t k = a.size();
  for (size_t i = 0; i < k; ++i) {
    const double r = (i > 0 ? std::sqrt(b2[i]) : 0.0) + (i + 1 < k ? std::sqrt(b2[i + 1]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_below(a, b2, mid) > idx)
      hi = mid;
    else
      lo = mid;
  }
  return 0.5 * (lo + hi);
}

static int quadratic_form_impl(const ld_csr* B, const double* x, void* stream, double* out) {
  int rc = check_csr(B, "B");
  if (rc) return rc;
  if (!out || (!x && B->rows > 0)) return fail(LD_EINVAL, "x or out is NULL");
  const int64_t d = B->rows;
  if (d == 0) {
    *out = 0.0;
    return LD_OK;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carve c;
  c.take((size_t)d * 8);
  c.take(kDotScratch * 8);
  c.take(8);
  Workspace ws;
  rc = get_workspace(nullptr, align_up(c.off), s, ws);
  if (rc) return rc;
  Carve cv;
  cv.base = static_cast<char*>(ws.ptr);
  double* y = static_cast<double*>(cv.take((size_t)d * 8));
  double* part = static_cast<double*>(cv.take(kDotScratch * 8));
  double* res = static_cast<double*>(cv.take(8));
  StepLaunch L{};
  L.nmat = 1;
  L.M = 1;
  L.shape = with_tile(base_shape(1, 1), d, B->nnz, 0);
  L.tile_rows = L.shape.tile_rows;
  L.ntiles = (d + L.tile_rows - 1) / L.tile_rows;
  StepDesc D{};
  D.row_ptr = B->row_ptr;
  D.col = B->col_idx;
  D.val = B->values;
  D.d = d;
  D.active = 1;
  D.G = x;
  D.out = y;
  D.ag = 1.0;
  D.bd = B->diag_shift;
  L.d0 = D;
  LD_HIP(launch_step(L, 1, valt_of(B->dtype), SRC_BUF, SRC_SAME, SRC_NONE, MU_NONE, s));  // y = (B + shift I) x
  LD_HIP(launch_dot(x, y, d, part, res, s));
  double h = 0.0;
  LD_HIP(hipMemcpyAsync(&h, res, 8, hipMemcpyDeviceToHost, s));
  LD_HIP(hipStreamSynchronize(s));
  *out = h;
  return LD_OK;
}

static int spectral_estimate_impl(const ld_csr* B, const ld_csr* Ct_in, int gram, int iters, uint64_t seed,
                                  void* stream, double* lo, double* hi) {
  int rc = check_csr(B, "B");
  if (rc) return rc;
  if (!lo || !hi) return fail(LD_EINVAL, "lo or hi is NULL");
  if (iters < 2 || iters > 2000) return fail(LD_EINVAL, "iters=%d out of range [2, 2000]", iters);
  if (B->rows < 1) return fail(LD_EINVAL, "empty matrix");
  if (gram && B->diag_shift != 0.0) return fail(LD_EINVAL, "diag_shift must be 0 with gram = 1");
  if (Ct_in) {
    rc = check_csr(Ct_in, "Ct");
    if (rc) return rc;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t d = B->rows;
  const int valt = valt_of(B->dtype);
  Carve c;
  for (int i = 0; i < 4; ++i) c.take((size_t)d * 8);
  c.take(kDotScratch * 8);
  c.take((size_t)iters * 8);  // alpha_j
  c.take((size_t)iters * 8);  // beta_j^2
  const bool build_t = gram && !Ct_in;
  if (build_t) {
    c.take((size_t)(d + 1) * 8);
    c.take((size_t)B->nnz * 4);
    c.take((size_t)B->nnz * val_bytes(valt));
    c.take((size_t)d * 8);
    c.take(transpose_scratch_bytes(d));
  }
  Workspace ws;
  rc = get_workspace(nullptr, align_up(c.off), s, ws);
  if (rc) return rc;
  Carve cv;
  cv.base = static_cast<char*>(ws.ptr);
  double* buf[3];
  for (auto& p : buf) p = static_cast<double*>(cv.take((size_t)d * 8));
  double* tmp = static_cast<double*>(cv.take((size_t)d * 8));
  double* part = static_cast<double*>(cv.take(kDotScratch * 8));
  double* al_dev = static_cast<double*>(cv.take((size_t)iters * 8));
  double* bb_dev = static_cast<double*>(cv.take((size_t)iters * 8));
  ld_csr Ct{};
  if (gram) {
    if (Ct_in) {
      Ct = *Ct_in;
    } else {
      int64_t* rpt = static_cast<int64_t*>(cv.take((size_t)(d + 1) * 8));
      int32_t* colt = static_cast<int32_t*>(cv.take((size_t)B->nnz * 4));
      void* valt_ = cv.take((size_t)B->nnz * val_bytes(valt));
      int64_t* cursor = static_cast<int64_t*>(cv.take((size_t)d * 8));
      void* scan = cv.take(transpose_scratch_bytes(d));
      LD_HIP(launch_transpose(B->row_ptr, B->col_idx, B->values, valt, d, B->nnz, rpt, colt, valt_, cursor, scan,
                              transpose_scratch_bytes(d), s));
      Ct = *B;
      Ct.row_ptr = rpt;
      Ct.col_idx = colt;
      Ct.values = valt_;
    }
  }
  // one-probe products in FP64 vectors through the recurrence-step kernel
  StepLaunch L{};
  L.nmat = 1;
  L.M = 1;
  L.shape = with_tile(base_shape(1, 1), d, B->nnz, 0);
  L.tile_rows = L.shape.tile_rows;
  L.ntiles = (d + L.tile_rows - 1) / L.tile_rows;
  auto product = [&](const ld_csr* X, const double* x, double* y, bool with_shift) -> hipError_t {
    StepDesc D{};
    D.row_ptr = X->row_ptr;
    D.col = X->col_idx;
    D.val = X->values;
    D.d = d;
    D.active = 1;
    D.G = x;
    D.out = y;
    D.ag = 1.0;
    D.bd = with_shift ? X->diag_shift : 0.0;
    L.d0 = D;
    return launch_step(L, 1, valt, SRC_BUF, with_shift ? SRC_SAME : SRC_NONE, SRC_NONE, MU_NONE, s);
  };
  double* vprev = buf[0];
  double* v = buf[1];
  double* w = buf[2];
  LD_HIP(launch_fill_zero(vprev, (size_t)d * 8, s));
  LD_HIP(launch_seed(v, 1, nullptr, nullptr, nullptr, 1.0 / std::sqrt((double)d), 0.0, 0.0, 0.0, seed, d, 1, s));
  // every step is queued at once: alpha_j and beta_j^2 stay in device memory (al_dev, bb_dev)
  // and the host reads them after the last step
  for (int j = 0; j < iters; ++j) {
    if (gram) {
      LD_HIP(product(B, v, tmp, false));
      LD_HIP(product(&Ct, tmp, w, false));
    } else {
      LD_HIP(product(B, v, w, true));
    }
    LD_HIP(launch_dot(w, v, d, part, al_dev + j, s));  // alpha_j = w^T v
    LD_HIP(launch_lanczos_update(w, v, vprev, al_dev + j, j > 0 ? bb_dev + j - 1 : nullptr, d, s));
    LD_HIP(launch_dot(w, w, d, part, bb_dev + j, s));   // beta_j^2
    LD_HIP(launch_lanczos_scale(w, bb_dev + j, d, vprev, s));  // v_{j+1} into the old v_{j-1} slot
    std::swap(vprev, v);                                       // v_{j-1} <- v_j, v_j <- v_{j+1}
  }
  std::vector<double> alh(iters), bbh(iters);
  LD_HIP(hipMemcpyAsync(alh.data(), al_dev, (size_t)iters * 8, hipMemcpyDeviceToHost, s));
  LD_HIP(hipMemcpyAsync(bbh.data(), bb_dev, (size_t)iters * 8, hipMemcpyDeviceToHost, s));
  LD_HIP(hipStreamSynchronize(s));
  // the tridiagonal matrix ends at the first step whose residual vanishes (an invariant subspace)
  // or breaks down; the steps queued after it only carried non-finite values
  std::vector<double> al, b2{0.0};
  for (int j = 0; j < iters; ++j) {
    al.push_back(alh[j]);
    if (!(bbh[j] > 0.0) || !std::isfinite(bbh[j])) break;
    if (j + 1 < iters) b2.push_back(bbh[j]);
  }
  b2.resize(al.size());
  *lo = tridiag_eig(al, b2, 0);
  *hi = tridiag_eig(al, b2, (int)al.size() - 1);
  return LD_OK;
}

static int clear_cache_impl(void) {
  {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    g_batch.clear();
  }
  {
    std::lock_guard<std::mutex> lk(g_pat_mu);
    g_pat.clear();
  }
  pool_release_all();
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  return LD_OK;
}

}  // extern "C"

// ======================================================================================
// C ABI: every entry point runs under `guarded`
// ======================================================================================

size_t ld_workspace_bytes(const ld_csr* B, int n, int M, int mode, int vec_f64) {
  return guarded<size_t>([&] { return workspace_bytes_impl(B, n, M, mode, vec_f64); });
}

int ld_logdet_cheb(const ld_csr* B, double a, double b, int n, int M, uint64_t seed, const ld_opts* opt,
                   void* stream, ld_result* out) {
  return guarded<int>([&] { return logdet_cheb_impl(B, a, b, n, M, seed, opt, stream, out); });
}

int ld_logdet_cheb_noalloc(const ld_csr* B, double a, double b, int n, int M, uint64_t seed, const ld_opts* opt,
                           void* stream, ld_result* out) {
  return guarded<int>([&] { return logdet_cheb_noalloc_impl(B, a, b, n, M, seed, opt, stream, out); });
}

int ld_logdet_taylor(const ld_csr* B, double a, double b, int n, int M, uint64_t seed, const ld_opts* opt,
                     void* stream, ld_result* out) {
  return guarded<int>([&] { return logdet_taylor_impl(B, a, b, n, M, seed, opt, stream, out); });
}

int ld_logabsdet_cheb(const ld_csr* C, const ld_csr* Ct, double smin, double smax, int n, int M, uint64_t seed,
                      const ld_opts* opt, void* stream, ld_result* out) {
  return guarded<int>([&] { return logabsdet_cheb_impl(C, Ct, smin, smax, n, M, seed, opt, stream, out); });
}

int ld_laplacian_minor(const ld_csr* adj, int64_t hub, int64_t* row_ptr_out, int32_t* col_out, void* val_out,
                       int32_t val_dtype, int64_t* max_degree, void* stream) {
  return guarded<int>([&] {
    return laplacian_minor_impl(adj, hub, row_ptr_out, col_out, val_out, val_dtype, max_degree, stream);
  });
}

int ld_log_spanning_trees(const ld_csr* adj, int64_t hub, int n, int M, uint64_t seed, int method, const ld_opts* opt,
                          void* stream, ld_result* out) {
  return guarded<int>([&] { return log_spanning_trees_impl(adj, hub, n, M, seed, method, opt, stream, out); });
}

int ld_gershgorin_batched(int count, const ld_csr* Bs, double* a, double* b, void* stream) {
  return guarded<int>([&] { return gershgorin_batched_impl(count, Bs, a, b, stream); });
}

int ld_gershgorin(const ld_csr* B, double* a, double* b, void* stream) {
  return guarded<int>([&] { return gershgorin_impl(B, a, b, stream); });
}

int ld_probes(uint64_t seed, int M, int64_t rows, int8_t* out, void* stream) {
  return guarded<int>([&] { return probes_impl(seed, M, rows, out, stream); });
}

int ld_transpose(const ld_csr* C, int64_t* row_ptr_t, int32_t* col_t, void* val_t, void* stream) {
  return guarded<int>([&] { return transpose_impl(C, row_ptr_t, col_t, val_t, stream); });
}

int ld_copy(void* dst, const void* src, size_t bytes, void* stream, double* ms) {
  return guarded<int>([&] { return copy_impl(dst, src, bytes, stream, ms); });
}

int ld_logdet_cheb_grad(const ld_csr* B, double a, double b, int n, int M, uint64_t seed, double grad_output,
                        void* grad_values, int grad_dtype, const ld_opts* opt, void* stream, ld_result* out) {
  return guarded<int>([&] {
    return logdet_cheb_grad_impl(B, a, b, n, M, seed, grad_output, grad_values, grad_dtype, opt, stream, out);
  });
}

int ld_logdet_cheb_batched(int count, const ld_csr* Bs, const double* a, const double* b, const int* n, int M,
                           uint64_t seed, const ld_opts* opt, void* stream, ld_result* outs) {
  return guarded<int>([&] { return logdet_cheb_batched_impl(count, Bs, a, b, n, M, seed, opt, stream, outs); });
}

int ld_quadratic_form(const ld_csr* B, const double* x, void* stream, double* out) {
  return guarded<int>([&] { return quadratic_form_impl(B, x, stream, out); });
}

int ld_spectral_estimate(const ld_csr* B, const ld_csr* Ct_in, int gram, int iters, uint64_t seed, void* stream,
                         double* lo, double* hi) {
  return guarded<int>([&] { return spectral_estimate_impl(B, Ct_in, gram, iters, seed, stream, lo, hi); });
}

int ld_clear_cache(void) {
  return guarded<int>([&] { return clear_cache_impl(); });
}
