// Host orchestration and the C ABI of libppca (see include/ppca.h).
//
// Each entry point validates its arguments, carves the caller's workspace
// into sub-buffers, enqueues the kernels of the step on the caller's stream,
// waits for the stream and returns the device status word.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <vector>

#include "ppca_common.h"

using namespace ppca;

// Fixed device scratch of ppca_rayleigh_ritz_noalloc: one copy per GPU the
// library runs on, held until the process ends, shared by every call on that
// GPU (calls that overlap on one GPU race on it).
constexpr size_t kStaticScratchBytes = PPCA_NOALLOC_SCRATCH_BYTES;
static_assert(kStaticScratchBytes % 256 == 0, "scratch size");
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

// ------------------------------------------------------------------ knobs
std::atomic<int64_t> g_chunk_rows{0};
std::atomic<int> g_fused_enabled{0};
constexpr int kFusedSpinLimit = 1 << 22;   // polls of one bounded wait (about 0.2 s)
std::mutex g_tmu;
bool g_timing = false;
struct KStat {
  int64_t launches = 0;
  double ms = 0.0;
};
KStat g_stats[6];
struct Pending {
  hipEvent_t a, b;
  int kernel;
};
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;

hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void resolve_timings() {
  std::lock_guard<std::mutex> lk(g_tmu);
  for (auto& p : g_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      g_stats[p.kernel].launches += 1;
      g_stats[p.kernel].ms += ms;
    }
    g_pool.push_back(p.a);
    g_pool.push_back(p.b);
  }
  g_pending.clear();
}

// Launch `f` bracketed by timing events when timing is on.
template <typename F>
hipError_t timed(int kernel, hipStream_t s, F&& f) {
  if (!g_timing) return f();
  hipEvent_t a, b;
  {
    std::lock_guard<std::mutex> lk(g_tmu);
    a = get_event();
    b = get_event();
  }
  if (!a || !b) return f();
  hipEventRecord(a, s);
  hipError_t e = f();
  hipEventRecord(b, s);
  std::lock_guard<std::mutex> lk(g_tmu);
  g_pending.push_back({a, b, kernel});
  return e;
}

// --------------------------------------------------------------- workspace
constexpr size_t kAlign = 256;

struct Carve {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off += (bytes + kAlign - 1) / kAlign * kAlign;
    return o;
  }
};

int elem_size(int32_t dtype) { return dtype == PPCA_F32 ? 4 : dtype == PPCA_BF16 ? 2 : 1; }

struct Plan {
  // dimensions
  int64_t n = 0, d = 0;
  int K = 0, Kp = 0;
  int64_t dp = 0;
  int64_t rows_cap = 0;   // rows of the Y staging buffer
  int ntiles = 0, nsplit = 0, ngpart = 0, ksplit = 1;
  bool fused = false;     // power passes (Z only) run the single-read kernel
  bool split = false;     // projection and Rayleigh-Ritz: two-term bf16 operand hi + lo
  int fnsplit = 0;
  size_t fex = 0, fyb = 0, fflags = 0, fdummy = 0, fpart = 0;
  // offsets
  size_t ypart = 0;
  size_t status = 0, vop = 0, rotp = 0, flip = 0, yb = 0, part = 0, gpart = 0, z = 0, g = 0, b = 0, gparts = 0,
         a = 0, rinv = 0, q1 = 0, t = 0, h = 0, w = 0, ev = 0, m = 0, egs = 0,
         sums = 0, cmax = 0, mean = 0, vprev = 0, chg = 0, su = 0, sw = 0, stmp = 0, sst = 0;
  size_t total = 0;
};

// Row splits of the X^T Y kernel: one workgroup per resident slot (the
// kernel's workgroups per CU times the CU count), at least 64 rows per split.
int nsplit_for(int ntiles, int Kp, int64_t rows) {
  int64_t ns = (int64_t)kNumCU * xty_blocks_per_cu(Kp) / ntiles;
  const int64_t by_rows = cdiv(rows, 64);
  if (ns > by_rows) ns = by_rows;
  if (ns < 1) ns = 1;
  return (int)ns;
}

Plan make_plan(int32_t op, int64_t n, int64_t d, int32_t dtype, int K, int64_t batch) {
  Plan p;
  p.n = n;
  p.d = d;
  p.K = K;
  p.Kp = (int)round_up(K, 16);
  p.dp = round_up(d, 64);   // whole 64-column k-steps of the streaming kernels
  // power and stream passes of bf16 data take the single-read pass, whose
  // products run on 32-column blocks: K is padded to 32 for the whole plan
  const int64_t chunk_knob = g_chunk_rows.load();
  const int64_t zrows = op == PPCA_OP_POWER ? n : batch;
  const bool fused = (op == PPCA_OP_POWER || op == PPCA_OP_STREAM) &&
                     g_fused_enabled.load() != 0 && K <= PPCA_MAX_K &&
                     fused_eligible(dtype, d, (int)round_up(K, 32)) &&
                     !(chunk_knob > 0 && chunk_knob < zrows);
  if (fused) p.Kp = (int)round_up(K, 32);
  // the projection of bf16 data and the Rayleigh-Ritz step that follows it
  // use the two-term operand (its products run on 32-column blocks)
  p.split = (op == PPCA_OP_PROJECT || op == PPCA_OP_RR) && dtype == PPCA_BF16;
  if (p.split) p.Kp = (int)round_up(K, 32);
  Carve c;
  p.status = c.take(256);
  if (op == PPCA_OP_CENTER) {
    const int nrb = prep_row_blocks(n);
    p.sums = c.take((size_t)nrb * d * 2 * sizeof(double));
    p.cmax = c.take((size_t)nrb * d * sizeof(float));
    p.mean = c.take((size_t)d * sizeof(double));
    p.total = c.off;
    return p;
  }
  const size_t kk = (size_t)K * K * sizeof(double);
  if (op == PPCA_OP_RR) {
    // the rotation reads V itself: no operand; per-workgroup column maxima
    // of the sign rule (rotate_blocks grows as k shrinks the tile's rows,
    // so K bounds every k <= K; at most 1024 workgroups, whatever d)
    p.rotp = c.take((size_t)rotate_blocks(d, K) * K * sizeof(ColMax));
    p.flip = c.take((size_t)K * sizeof(int));
    p.rinv = c.take(kk);
    p.t = c.take(kk);
    p.h = c.take(kk);
    p.w = c.take(kk);
    p.ev = c.take((size_t)K * sizeof(double));
    p.m = c.take(kk);
    p.total = c.off;
    return p;
  }
  const int es_op = dtype == PPCA_F32 ? 4 : 2;
  p.vop = c.take((size_t)p.Kp * p.dp * es_op * (p.split ? 2 : 1));
  int64_t pass_rows = n;
  if (op == PPCA_OP_OJA || op == PPCA_OP_EIGENGAME || op == PPCA_OP_STREAM) pass_rows = batch;
  if (op == PPCA_OP_PROJECT && batch > 0) pass_rows = batch;   // projection of a row window
  const int64_t chunk = g_chunk_rows.load();
  if (chunk > 0 && chunk < pass_rows) pass_rows = round_up(chunk, 256);
  p.rows_cap = round_up(pass_rows, 256);
  const int es_y = dtype == PPCA_F32 ? 4 : 2;
  // the projection pass keeps Y on chip (only G = Y^T Y is needed)
  p.yb = c.take(op == PPCA_OP_PROJECT ? 16 : (size_t)p.rows_cap * p.Kp * es_y);
  // the Gram-only pass (projection) runs no X^T Y kernel
  p.ntiles = xty_tiles(d, p.Kp);
  p.nsplit = nsplit_for(p.ntiles, p.Kp, p.rows_cap);
  p.part = c.take(op == PPCA_OP_PROJECT
                      ? 16
                      : (size_t)p.ntiles * p.nsplit * p.Kp * xty_cols(p.Kp) * sizeof(float));
  // the two-term projection: column split on short passes (as every short
  // pass), else k_xvg (one partial per workgroup)
  p.ksplit = xv_ksplit(dtype, p.Kp, d, p.rows_cap);
  p.ngpart = (p.split && p.ksplit == 1) ? xvg_grid(p.rows_cap) : xv_grid(dtype, p.Kp, d, p.rows_cap);
  p.gpart = c.take((size_t)p.ngpart * p.Kp * p.Kp * sizeof(float));
  p.ypart = c.take(p.ksplit > 1 ? (size_t)p.ksplit * round_up(p.rows_cap, 64) * p.Kp * sizeof(float)
                                : 16);
  p.z = c.take((size_t)d * K * sizeof(float));
  p.g = c.take(kk);
  p.b = c.take(kk);
  p.gparts = c.take((size_t)gram_parts(d, K) * K * K * sizeof(double));
  p.a = c.take(kk);
  p.rinv = c.take(kk);
  p.q1 = c.take((size_t)d * K * sizeof(double));
  if (fused) {
    const FusedSizes fz = fused_sizes(d, p.Kp);
    p.fused = true;
    p.fnsplit = fz.nsplit;
    p.fex = c.take(fz.ex_bytes);
    p.fyb = c.take(fz.yb_bytes);
    p.fflags = c.take(fz.flag_bytes);
    p.fdummy = c.take(fz.dummy_bytes);
    p.fpart = c.take(fz.part_bytes);
  }
  if (op == PPCA_OP_POWER) {
    p.vprev = c.take((size_t)d * K * sizeof(float));   // termination rule: previous iterate
    p.chg = c.take((size_t)K * sizeof(double));        // ... and the span change per column
  }
  if (op == PPCA_OP_EIGENGAME) {
    p.egs = c.take(eigengame_scratch_doubles(d, K) * sizeof(double));
  }
  p.total = c.off;
  return p;
}

// Sequential power method: the plan of a K = 1 power pass, then three
// d-vectors and the step state of the direction being computed.
Plan make_seq_plan(int64_t n, int64_t d, int32_t dtype) {
  Plan p = make_plan(PPCA_OP_POWER, n, d, dtype, 1, 0);
  Carve c;
  c.off = p.total;
  p.su = c.take((size_t)d * sizeof(float));
  p.sw = c.take((size_t)d * sizeof(float));
  p.stmp = c.take((size_t)d * sizeof(float));
  p.sst = c.take(256);
  p.total = c.off;
  return p;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(ws) + off);
}

// ------------------------------------------------------------- validation
int check_matrix(const ppca_matrix* X) {
  if (!X || !X->x) return PPCA_ERR_ARG;
  if (X->n < 1 || X->d < 1 || X->ld < X->d) return PPCA_ERR_ARG;
  if (X->dtype != PPCA_F32 && X->dtype != PPCA_BF16 && X->dtype != PPCA_FP8_E4M3)
    return PPCA_ERR_DTYPE;
  if ((X->dtype == PPCA_FP8_E4M3) != (X->col_scale != nullptr)) return PPCA_ERR_DTYPE;
  const int es = elem_size(X->dtype);
  if ((reinterpret_cast<uintptr_t>(X->x) % 16) != 0 || ((X->ld * es) % 16) != 0)
    return PPCA_ERR_ALIGN;
  return PPCA_OK;
}

int check_k(const ppca_matrix* X, int K) {
  if (K < 1 || K > PPCA_MAX_K || K > X->d || K > X->n) return PPCA_ERR_ARG;
  return PPCA_OK;
}

int check_ws(void* ws, size_t ws_bytes, const Plan& p) {
  if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0 || ws_bytes < p.total)
    return PPCA_ERR_WORKSPACE;
  return PPCA_OK;
}

#define HIP_TRY(expr)                          \
  do {                                         \
    if ((expr) != hipSuccess) return PPCA_ERR_HIP; \
  } while (0)

int finish(const Plan& p, void* ws, hipStream_t s) {
  int h = 0;
  if (hipMemcpyAsync(&h, at<int>(ws, p.status), sizeof(int), hipMemcpyDeviceToHost, s) !=
      hipSuccess)
    return PPCA_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return PPCA_ERR_HIP;
  if (g_timing) resolve_timings();
  return h;
}

// ------------------------------------------------------------ building blocks
StreamBufs bufs_of(const Plan& p, void* ws) {
  StreamBufs b;
  b.vop = at<void>(ws, p.vop);
  b.dp = p.dp;
  b.yb = at<void>(ws, p.yb);
  b.part = at<float>(ws, p.part);
  b.gpart = at<float>(ws, p.gpart);
  b.rows_cap = p.rows_cap;
  b.nsplit = p.nsplit;
  b.ngpart = p.ngpart;
  b.Kp = p.Kp;
  b.ksplit = p.ksplit;
  b.ypart = at<float>(ws, p.ypart);
  b.split = p.split;
  return b;
}

// One streaming pass over rows r0 .. r0+nrows-1 (mod n): Z (unless gram_only) and
// G (when G is not null).
int run_pass(const ppca_matrix* X, const Plan& p, void* ws, int64_t r0, int64_t nrows, float* Z,
             double* G, double* Gcopy, bool gram_only, hipStream_t s) {
  PassDesc pd;
  pd.x = X->x;
  pd.n = X->n;
  pd.d = X->d;
  pd.ld = X->ld;
  pd.dtype = X->dtype;
  pd.col_scale = X->col_scale;
  pd.r0 = r0;
  pd.nrows = nrows;
  StreamBufs b = bufs_of(p, ws);
  if (p.fused && !gram_only && G == nullptr) {
    // Z = X^T bf16(X V') in one read of X, then the fixed-order float64 sum of
    // the (slice, cluster) partials
    FusedBufs fb{at<float>(ws, p.fex), at<uint16_t>(ws, p.fyb), at<int>(ws, p.fflags),
                 at<float>(ws, p.fdummy), at<float>(ws, p.fpart)};
    HIP_TRY(timed(3, s, [&] {
      return launch_fused_pass(pd, b.vop, b.dp, p.Kp, fb, at<int>(ws, p.status), kFusedSpinLimit,
                               s);
    }));
    StreamBufs bz = b;
    bz.part = fb.part;
    bz.nsplit = p.fnsplit;
    HIP_TRY(launch_reduce_zg(bz, X->d, p.K, nullptr, Z, nullptr, nullptr, false,
                             at<int>(ws, p.status), s));
    return PPCA_OK;
  }
  const int64_t chunk = (p.rows_cap < nrows) ? p.rows_cap : nrows;
  // one row split and one chunk: the X^T Y kernel writes Z itself
  const bool direct_z = !gram_only && p.nsplit == 1 && nrows <= chunk;
  int* st = at<int>(ws, p.status);
  for (int64_t i0 = 0; i0 < nrows; i0 += chunk) {
    const int64_t rows = (nrows - i0) < chunk ? (nrows - i0) : chunk;
    HIP_TRY(timed(gram_only ? 4 : 0, s, [&] {
      return launch_xv(pd, b, i0, rows, !gram_only, G != nullptr, i0 > 0, s);
    }));
    if (!gram_only)
      HIP_TRY(timed(1, s, [&] {
        return launch_xty(pd, b, i0, rows, i0 > 0, direct_z ? Z : nullptr, p.K, st, s);
      }));
  }
  HIP_TRY(launch_reduce_zg(b, X->d, p.K, X->dtype == PPCA_FP8_E4M3 ? X->col_scale : nullptr, Z, G,
                           Gcopy, gram_only || direct_z, st, s));
  return PPCA_OK;
}

// V (d x K f32) <- CholQR2(A) for A (d x K f32); A and V may alias.
int cholqr2(const float* A, float* V, int64_t d, int K, const Plan& p, void* ws, hipStream_t s) {
  int* st = at<int>(ws, p.status);
  double* gp = at<double>(ws, p.gparts);
  double* Am = at<double>(ws, p.a);
  double* Ri = at<double>(ws, p.rinv);
  double* Q1 = at<double>(ws, p.q1);
  HIP_TRY(launch_gram(A, false, d, K, K, gp, Am, st, s));
  HIP_TRY(launch_chol_inv(Am, K, nullptr, Ri, st, s));
  HIP_TRY(launch_trmm(A, false, d, K, K, Ri, Q1, true, K, st, s));
  HIP_TRY(launch_gram(Q1, true, d, K, K, gp, Am, st, s));
  HIP_TRY(launch_chol_inv(Am, K, nullptr, Ri, st, s));
  HIP_TRY(launch_trmm(Q1, true, d, K, K, Ri, V, false, K, st, s));
  return PPCA_OK;
}

int make_operand(const ppca_matrix* X, const float* V, const Plan& p, void* ws, hipStream_t s) {
  HIP_TRY(launch_make_operand(V, X->d, p.K, p.Kp, p.dp, X->dtype, X->col_scale,
                              at<void>(ws, p.vop), p.split, s));
  return PPCA_OK;
}

// B = V_eff^T V_eff (K x K f64), V_eff the operand's values, recomputed from V
int operand_gram(const ppca_matrix* X, const float* V, const Plan& p, void* ws, double* B,
                 hipStream_t s) {
  HIP_TRY(launch_operand_gram(V, X->d, p.K, X->dtype, p.split, X->col_scale,
                              at<double>(ws, p.gparts), B, at<int>(ws, p.status), s));
  return PPCA_OK;
}

#define RET_IF(expr)            \
  do {                          \
    const int _rc = (expr);     \
    if (_rc != PPCA_OK) return _rc; \
  } while (0)


int check_rr(const ppca_matrix* X, int K, int k, const double* G, const double* B,
             const float* V, const float* E, const double* evals) {
  if (!X || X->n < 1 || X->d < 1) return PPCA_ERR_ARG;
  if (X->dtype != PPCA_F32 && X->dtype != PPCA_BF16 && X->dtype != PPCA_FP8_E4M3)
    return PPCA_ERR_DTYPE;
  if ((X->dtype == PPCA_FP8_E4M3) != (X->col_scale != nullptr)) return PPCA_ERR_DTYPE;
  if (K < 1 || K > PPCA_MAX_K || K > X->d || k < 1 || k > K) return PPCA_ERR_ARG;
  if (!G || !B || !evals || (E && !V)) return PPCA_ERR_ARG;
  return PPCA_OK;
}

// Rayleigh-Ritz (Alg. 1 step 4) on a validated workspace of plan p.
int rayleigh_ritz_on(const ppca_matrix* X, int K, int k, const double* G, const double* B,
                     const float* V, float* E, double* evals, const Plan& p, void* ws,
                     hipStream_t s) {
  int* st = at<int>(ws, p.status);
  HIP_TRY(launch_zero(st, 256, s));
  double* Ri = at<double>(ws, p.rinv);
  double* T = at<double>(ws, p.t);
  double* H = at<double>(ws, p.h);
  double* W = at<double>(ws, p.w);
  double* ev = at<double>(ws, p.ev);
  double* M = at<double>(ws, p.m);
  HIP_TRY(launch_chol_inv(B, K, nullptr, Ri, st, s));
  HIP_TRY(launch_small_gemm(G, false, Ri, T, K, K, K, K, K, K, 1.0, st, s));
  HIP_TRY(launch_small_gemm(Ri, true, T, H, K, K, K, K, K, K, 1.0 / (double)X->n, st, s));
  HIP_TRY(launch_jacobi(H, K, W, ev, 60, st, s));
  HIP_TRY(launch_copy_f64(ev, evals, k, s));
  if (E) {
    HIP_TRY(launch_small_gemm(Ri, false, W, M, K, k, K, K, K, k, 1.0, st, s));
    HIP_TRY(launch_rotate(V, X->d, K, X->dtype, p.split, X->col_scale, M, k, E,
                          at<ColMax>(ws, p.rotp), at<int>(ws, p.flip), st, s));
  }
  return finish(p, ws, s);
}

// ------------------------------------------------------- fixed device scratch
// Per-device address of the file-scope scratch array (host code must not
// pass the array's own name to a kernel: on the host it is only a stand-in
// for the symbol).  Looked up once per device, with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int static_scratch(hipStream_t s, void** out) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur < 0 || cur >= kMaxDevices) return PPCA_ERR_HIP;
  hipDevice_t sdev = -1;
  if (hipStreamGetDevice(s, &sdev) != hipSuccess) return PPCA_ERR_HIP;
  if (sdev != cur) return PPCA_ERR_ARG;   // the stream must belong to the current device
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[cur]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
      return PPCA_ERR_HIP;
    if ((reinterpret_cast<uintptr_t>(ptr) % kAlign) != 0) return PPCA_ERR_HIP;
    g_scratch_ptr[cur] = ptr;
  }
  *out = g_scratch_ptr[cur];
  return PPCA_OK;
}

// ---------------------------------------------------------- grouped problems
constexpr int64_t kGroupItemBytes = 3 << 20;   // X bytes per work item (default target)
constexpr int64_t kGroupItemMin = 1 << 16, kGroupItemMax = 1LL << 30;
std::atomic<int64_t> g_group_item_bytes{kGroupItemBytes};

struct GroupPlan {
  size_t status = 0, probs = 0, items = 0, blk_z = 0, blk_g = 0, order = 0, zpart = 0, gpart = 0;
  size_t total = 0;
  std::vector<GProb> hp;
  std::vector<GItem> hi;
  std::vector<int> bz, bg;                       // reduce block starts, nprob + 1 each
  std::vector<int> ord;                          // problems by d K^2, largest first
  std::vector<size_t> pv, pz, pq, pk;            // per problem: vop, Z, q1, K x K block
};

int check_group_problem(const ppca_problem& q) {
  const int rc = check_matrix(&q.X);
  if (rc != PPCA_OK) return rc;
  if (q.X.dtype != PPCA_BF16) return PPCA_ERR_DTYPE;
  if (q.X.d > kGroupMaxD || q.X.ld > kGroupMaxLd || q.k < 1 || q.l < 0) return PPCA_ERR_ARG;
  const int64_t K = (int64_t)q.k + q.l;
  if (K > kGroupMaxK || K > q.X.d || K > q.X.n) return PPCA_ERR_ARG;
  return PPCA_OK;
}

int make_group_plan(const ppca_problem* pr, int nprob, GroupPlan& gp,
                    int64_t item_bytes = g_group_item_bytes.load()) {
  if (!pr || nprob < 1) return PPCA_ERR_ARG;
  Carve c;
  gp.status = c.take(256);
  gp.hp.assign(nprob, GProb{});
  gp.bz.assign(nprob + 1, 0);
  gp.bg.assign(nprob + 1, 0);
  gp.pv.resize(nprob);
  gp.pz.resize(nprob);
  gp.pq.resize(nprob);
  gp.pk.resize(nprob);
  gp.hi.clear();
  int64_t zf = 0, gf = 0;
  for (int p = 0; p < nprob; ++p) {
    const ppca_problem& q = pr[p];
    const int rc = check_group_problem(q);
    if (rc != PPCA_OK) return rc;
    const int64_t n = q.X.n, d = q.X.d;
    const int K = q.k + q.l, Kp = (int)round_up(K, 32);
    const int dci = group_dci(d), dc = group_class_width(dci), wr = group_row_groups(dci);
    GProb& P = gp.hp[p];
    P.x = reinterpret_cast<const uint16_t*>(q.X.x);
    P.n = n;
    P.d = d;
    P.ld = q.X.ld;
    P.K = K;
    P.Kp = Kp;
    P.k = q.k;
    P.cls = dci * 2 + Kp / 32 - 1;
    P.dc = dc;
    P.wr = wr;
    // work items: about item_bytes of X each, whole 16-row tiles of every row group
    const int64_t step = 16 * wr;
    int64_t rt = round_up(std::max<int64_t>(cdiv(item_bytes, d * 2), step), step);
    int64_t ni = cdiv(n, rt);
    rt = round_up(cdiv(n, ni), step);
    ni = cdiv(n, rt);
    P.nitem = (int32_t)ni;
    P.zbase = zf;
    P.gbase = gf;
    const int64_t zs = (int64_t)wr * Kp * dc, gs = (int64_t)4 * Kp * Kp;
    for (int64_t m = 0; m < ni; ++m) {
      GItem it{};
      it.prob = p;
      it.r0 = m * rt;
      it.rows = std::min(rt, n - m * rt);
      it.zoff = zf + m * zs;
      it.goff = gf + m * gs;
      gp.hi.push_back(it);
    }
    zf += ni * zs;
    gf += ni * gs;
    gp.bz[p + 1] = gp.bz[p] + (int)cdiv(d * K, 256);
    gp.bg[p + 1] = gp.bg[p] + (int)cdiv((int64_t)K * K, 256);
    const size_t kk = (size_t)K * K * sizeof(double);
    gp.pv[p] = c.take((size_t)2 * Kp * dc * sizeof(uint16_t));   // hi, then lo
    gp.pz[p] = c.take((size_t)d * K * sizeof(float));
    gp.pq[p] = c.take((size_t)d * K * sizeof(double));
    gp.pk[p] = c.take(5 * kk + (size_t)K * sizeof(double));
  }
  // Order of the items, which workgroup w of the pass takes at positions w,
  // w + G, w + 2G, ... (G = min(items, CUs)).  Largest estimated cost first:
  // X bytes, times 1.2 for Kp = 64, whose MFMA work doubles (the measured rate
  // per class is about 5.4 TB/s at Kp = 32 and 4.5 at Kp = 64); ties by
  // problem and row, so the order is fixed.  Then every second round of G
  // items is reversed, so that the workgroups taking the largest item of one
  // round take the smallest of the next.  Results do not depend on this
  // order: an item's partial slot and the order of the reduction follow its
  // position within its problem.
  auto cost = [&](const GItem& a) {
    const GProb& P = gp.hp[a.prob];
    return (a.rows * P.d) * (P.Kp > 32 ? 6 : 5);
  };
  std::stable_sort(gp.hi.begin(), gp.hi.end(),
                   [&](const GItem& a, const GItem& b) { return cost(a) > cost(b); });
  {
    const size_t G = std::min<size_t>(gp.hi.size(), (size_t)kNumCU);
    for (size_t r0 = G; r0 < gp.hi.size(); r0 += 2 * G)
      std::reverse(gp.hi.begin() + r0, gp.hi.begin() + std::min(gp.hi.size(), r0 + G));
  }
  gp.ord.resize(nprob);
  for (int p = 0; p < nprob; ++p) gp.ord[p] = p;
  std::stable_sort(gp.ord.begin(), gp.ord.end(), [&](int a, int b) {
    const GProb &A = gp.hp[a], &B = gp.hp[b];
    return A.d * A.K * A.K > B.d * B.K * B.K;
  });
  gp.probs = c.take(gp.hp.size() * sizeof(GProb));
  gp.items = c.take(gp.hi.size() * sizeof(GItem));
  gp.blk_z = c.take(gp.bz.size() * sizeof(int));
  gp.blk_g = c.take(gp.bg.size() * sizeof(int));
  gp.order = c.take(gp.ord.size() * sizeof(int));
  gp.zpart = c.take((size_t)zf * sizeof(float));
  gp.gpart = c.take((size_t)gf * sizeof(float));
  gp.total = c.off;
  return PPCA_OK;
}

// Device pointers of the per-problem buffers and the caller's arrays.
void bind_group_plan(GroupPlan& gp, const ppca_problem* pr, void* ws) {
  for (size_t p = 0; p < gp.hp.size(); ++p) {
    GProb& P = gp.hp[p];
    const ppca_problem& q = pr[p];
    P.V = q.V;
    P.G = q.G;
    P.B = q.B;
    P.E = q.E;
    P.evals = q.evals;
    P.vop = at<uint16_t>(ws, gp.pv[p]);
    P.vlo = P.vop + (size_t)P.Kp * P.dc;
    P.Z = at<float>(ws, gp.pz[p]);
    P.q1 = at<double>(ws, gp.pq[p]);
    double* kb = at<double>(ws, gp.pk[p]);
    const size_t kk = (size_t)P.K * P.K;
    P.A = kb;
    P.R = kb + kk;
    P.Rinv = kb + 2 * kk;
    P.H = kb + 3 * kk;
    P.W = kb + 4 * kk;
    P.ev = kb + 5 * kk;
  }
}

int upload_group_plan(const GroupPlan& gp, void* ws, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(at<void>(ws, gp.probs), gp.hp.data(), gp.hp.size() * sizeof(GProb),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(at<void>(ws, gp.items), gp.hi.data(), gp.hi.size() * sizeof(GItem),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(at<void>(ws, gp.blk_z), gp.bz.data(), gp.bz.size() * sizeof(int),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(at<void>(ws, gp.blk_g), gp.bg.data(), gp.bg.size() * sizeof(int),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(at<void>(ws, gp.order), gp.ord.data(), gp.ord.size() * sizeof(int),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(launch_zero(at<int>(ws, gp.status), 256, s));
  return PPCA_OK;
}

int finish_group(const GroupPlan& gp, void* ws, hipStream_t s) {
  int h = 0;
  if (hipMemcpyAsync(&h, at<int>(ws, gp.status), sizeof(int), hipMemcpyDeviceToHost, s) !=
      hipSuccess)
    return PPCA_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return PPCA_ERR_HIP;
  if (g_timing) resolve_timings();
  return h;
}

int check_group_ws(void* ws, size_t ws_bytes, const GroupPlan& gp) {
  if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0 || ws_bytes < gp.total)
    return PPCA_ERR_WORKSPACE;
  return PPCA_OK;
}

// One power iteration of every problem: fused Z pass, reduction, CholeskyQR2.
int group_iteration(const GroupPlan& gp, void* ws, bool want_b, bool time_it, hipStream_t s) {
  const GProb* dP = at<GProb>(ws, gp.probs);
  const int nprob = (int)gp.hp.size(), nitems = (int)gp.hi.size();
  const int grid = std::min(nitems, kNumCU);
  int* st = at<int>(ws, gp.status);
  auto pass = [&] {
    return launch_group_pass(dP, at<GItem>(ws, gp.items), nitems, grid, at<float>(ws, gp.zpart),
                             at<float>(ws, gp.gpart), true, s);
  };
  HIP_TRY(time_it ? timed(2, s, pass) : pass());
  HIP_TRY(launch_group_reduce(dP, nprob, at<int>(ws, gp.blk_z), gp.bz.back(),
                              at<float>(ws, gp.zpart), at<float>(ws, gp.gpart), true, st, s));
  HIP_TRY(launch_group_cholqr2(dP, at<int>(ws, gp.order), nprob, false, want_b, st, s));
  return PPCA_OK;
}
int check_sgd(const ppca_matrix* X, const ppca_sgd_params* q) {
  if (!q) return PPCA_ERR_ARG;
  if (q->batch < 1 || q->batch > X->n || q->steps < 0 || q->start_step < 0) return PPCA_ERR_ARG;
  if (!(q->eta0 > 0.0) || !isfinite(q->eta0) || !isfinite(q->t0)) return PPCA_ERR_ARG;
  if (!(q->momentum >= 0.0 && q->momentum < 1.0)) return PPCA_ERR_ARG;
  if (q->momentum > 0.0 && !q->mom_buf) return PPCA_ERR_ARG;
  if (q->nesterov != 0 && q->nesterov != 1) return PPCA_ERR_ARG;
  if (q->snapshot_every < 0) return PPCA_ERR_ARG;
  if (q->snapshot_every > 0 && !q->snapshots) return PPCA_ERR_ARG;
  return PPCA_OK;
}

int prime_sgd(bool eigengame, const ppca_matrix* X, int32_t k, int32_t l, const ppca_sgd_params* q,
              float* V, void* ws, size_t ws_bytes, void* stream) {
  RET_IF(check_matrix(X));
  if (k < 1 || l < 0 || !V) return PPCA_ERR_ARG;
  const int K = k + l;
  RET_IF(check_k(X, K));
  RET_IF(check_sgd(X, q));
  const Plan p = make_plan(eigengame ? PPCA_OP_EIGENGAME : PPCA_OP_OJA, X->n, X->d, X->dtype, K,
                           q->batch);
  RET_IF(check_ws(ws, ws_bytes, p));
  hipStream_t s = (hipStream_t)stream;
  int* st = at<int>(ws, p.status);
  HIP_TRY(launch_zero(st, 256, s));
  if (q->orthonormalise_start) RET_IF(cholqr2(V, V, X->d, K, p, ws, s));
  float* Z = at<float>(ws, p.z);
  double* G = at<double>(ws, p.g);
  const int64_t b = q->batch;
  for (int64_t t = 0; t < q->steps; ++t) {
    const int64_t gstep = q->start_step + t;
    const int64_t r0 = (int64_t)(((__int128)gstep * b) % X->n);
    // each update writes the next step's operand itself
    if (t == 0) RET_IF(make_operand(X, V, p, ws, s));
    RET_IF(run_pass(X, p, ws, r0, b, Z, G, nullptr, false, s));
    const double eta = q->t0 > 0.0 ? q->eta0 / (1.0 + (double)gstep / q->t0) : q->eta0;
    void* next_op = t + 1 < q->steps ? at<void>(ws, p.vop) : nullptr;
    if (eigengame) {
      HIP_TRY(launch_eigengame_update(V, Z, G, X->d, K, (int)b, eta, q->momentum, q->nesterov,
                                      q->mom_buf, at<double>(ws, p.egs), next_op, p.dp, X->dtype,
                                      X->col_scale, st, s));
    } else {
      HIP_TRY(launch_sanger_update(V, Z, G, X->d, K, (int)b, eta, q->momentum, q->nesterov,
                                   q->mom_buf, next_op, p.dp, X->dtype, X->col_scale, st, s));
    }
    if (q->snapshot_every > 0 && (t + 1) % q->snapshot_every == 0) {
      const int64_t slot = (t + 1) / q->snapshot_every - 1;
      HIP_TRY(launch_copy_f32(V, q->snapshots + slot * X->d * K, X->d * K, s));
    }
  }
  return finish(p, ws, s);
}

}  // namespace

extern "C" {

int ppca_center_quantize(const float* x, int64_t n, int64_t d, int64_t ldx, int32_t out_dtype,
                         void* out, int64_t ldo, float* col_scale, double* mean, void* ws,
                         size_t ws_bytes, void* stream) {
  if (!x || !out || n < 1 || d < 1 || ldx < d || ldo < d) return PPCA_ERR_ARG;
  if (out_dtype != PPCA_F32 && out_dtype != PPCA_BF16 && out_dtype != PPCA_FP8_E4M3)
    return PPCA_ERR_DTYPE;
  if ((out_dtype == PPCA_FP8_E4M3) != (col_scale != nullptr)) return PPCA_ERR_DTYPE;
  const bool same = (const void*)x == (const void*)out;
  if (same && !(out_dtype == PPCA_F32 && ldx == ldo)) return PPCA_ERR_ARG;
  const Plan p = make_plan(PPCA_OP_CENTER, n, d, out_dtype, 1, 0);
  RET_IF(check_ws(ws, ws_bytes, p));
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_zero(at<int>(ws, p.status), 256, s));
  HIP_TRY(launch_center_quantize(x, n, d, ldx, out_dtype, out, ldo, col_scale, mean,
                                 at<double>(ws, p.sums), at<float>(ws, p.cmax),
                                 at<double>(ws, p.mean), s));
  return finish(p, ws, s);
}

int ppca_prime_power(const ppca_matrix* X, int32_t k, int32_t l, int32_t iters, float* V,
                     double* gram_hist, double* b_hist, void* ws, size_t ws_bytes, void* stream) {
  RET_IF(check_matrix(X));
  if (k < 1 || l < 0 || iters < 0 || !V) return PPCA_ERR_ARG;
  const int K = k + l;
  RET_IF(check_k(X, K));
  const Plan p = make_plan(PPCA_OP_POWER, X->n, X->d, X->dtype, K, 0);
  RET_IF(check_ws(ws, ws_bytes, p));
  hipStream_t s = (hipStream_t)stream;
  int* st = at<int>(ws, p.status);
  HIP_TRY(launch_zero(st, 256, s));
  RET_IF(cholqr2(V, V, X->d, K, p, ws, s));
  float* Z = at<float>(ws, p.z);
  double* G = at<double>(ws, p.g);
  const int64_t kk = (int64_t)K * K;
  for (int t = 0; t < iters; ++t) {
    RET_IF(make_operand(X, V, p, ws, s));
    if (b_hist) RET_IF(operand_gram(X, V, p, ws, b_hist + t * kk, s));
    // G = Y^T Y is only formed when the caller asks for its history
    RET_IF(run_pass(X, p, ws, 0, X->n, Z, gram_hist ? G : nullptr,
                    gram_hist ? gram_hist + t * kk : nullptr, false, s));
    RET_IF(cholqr2(Z, V, X->d, K, p, ws, s));
  }
  return finish(p, ws, s);
}

int ppca_prime_power_eps(const ppca_matrix* X, int32_t k, int32_t l, int32_t max_iters, double eps,
                         float* V, int32_t* iters_done, double* changes, void* ws,
                         size_t ws_bytes, void* stream) {
  RET_IF(check_matrix(X));
  if (k < 1 || l < 0 || max_iters < 1 || !V || !iters_done) return PPCA_ERR_ARG;
  if (!(eps >= 0.0) || !isfinite(eps)) return PPCA_ERR_ARG;
  const int K = k + l;
  RET_IF(check_k(X, K));
  const Plan p = make_plan(PPCA_OP_POWER, X->n, X->d, X->dtype, K, 0);
  RET_IF(check_ws(ws, ws_bytes, p));
  hipStream_t s = (hipStream_t)stream;
  int* st = at<int>(ws, p.status);
  HIP_TRY(launch_zero(st, 256, s));
  RET_IF(cholqr2(V, V, X->d, K, p, ws, s));
  float* Z = at<float>(ws, p.z);
  float* Vp = at<float>(ws, p.vprev);
  double* ch = at<double>(ws, p.chg);
  *iters_done = max_iters;
  for (int t = 1; t <= max_iters; ++t) {
    HIP_TRY(launch_copy_f32(V, Vp, X->d * K, s));
    RET_IF(make_operand(X, V, p, ws, s));
    RET_IF(run_pass(X, p, ws, 0, X->n, Z, nullptr, nullptr, false, s));
    RET_IF(cholqr2(Z, V, X->d, K, p, ws, s));
    HIP_TRY(launch_span_change(V, Vp, X->d, K, ch, s));
    double hres[PPCA_MAX_K];
    int hst = 0;
    HIP_TRY(hipMemcpyAsync(hres, ch, (size_t)K * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&hst, st, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hst != PPCA_OK) return hst;
    double h = 0.0;
    for (int j = 0; j < K; ++j) h = hres[j] > h ? hres[j] : h;
    if (changes) changes[t - 1] = h;
    if (h < eps) {
      *iters_done = t;
      break;
    }
  }
  return finish(p, ws, s);
}

int ppca_prime_power_seq(const ppca_matrix* X, int32_t k, int32_t l, double eps,
                         int32_t max_steps, float* V, int32_t* steps, void* ws, size_t ws_bytes,
                         void* stream) {
  RET_IF(check_matrix(X));
  if (k < 1 || l < 0 || max_steps < 1 || !V || !steps) return PPCA_ERR_ARG;
  if (!(eps >= 0.0) || !isfinite(eps)) return PPCA_ERR_ARG;
  const int K = k + l;
  RET_IF(check_k(X, K));
  const Plan p = make_seq_plan(X->n, X->d, X->dtype);
  RET_IF(check_ws(ws, ws_bytes, p));
  hipStream_t s = (hipStream_t)stream;
  int* st = at<int>(ws, p.status);
  HIP_TRY(launch_zero(st, 256, s));
  float* u = at<float>(ws, p.su);
  float* w = at<float>(ws, p.sw);
  float* tmp = at<float>(ws, p.stmp);
  SeqState* ss = at<SeqState>(ws, p.sst);
  float* Z = at<float>(ws, p.z);
  constexpr int kBatch = 8;   // steps between two reads of the state
  for (int i = 0; i < K; ++i) {
    HIP_TRY(launch_seq_start(V, X->d, K, i, u, ss, tmp, st, s));
    SeqState h{0, 0, 0.0};
    while (!h.done) {
      for (int b = 0; b < kBatch; ++b) {
        // Z = X^T X u: the power step's pass with K = 1 (u is a d x 1 block)
        RET_IF(make_operand(X, u, p, ws, s));
        RET_IF(run_pass(X, p, ws, 0, X->n, Z, nullptr, nullptr, false, s));
        HIP_TRY(launch_seq_step(V, X->d, K, i, Z, u, w, ss, eps, max_steps, st, s));
      }
      int hst = 0;
      HIP_TRY(hipMemcpyAsync(&h, ss, sizeof(SeqState), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(&hst, st, sizeof(int), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (hst != PPCA_OK) return hst;
    }
    HIP_TRY(launch_seq_store(V, X->d, K, i, u, s));
    steps[i] = h.steps;
  }
  return finish(p, ws, s);
}

int ppca_prime_oja(const ppca_matrix* X, int32_t k, int32_t l, const ppca_sgd_params* p, float* V,
                   void* ws, size_t ws_bytes, void* stream) {
  return prime_sgd(false, X, k, l, p, V, ws, ws_bytes, stream);
}

int ppca_prime_eigengame(const ppca_matrix* X, int32_t k, int32_t l, const ppca_sgd_params* p,
                         float* V, void* ws, size_t ws_bytes, void* stream) {
  return prime_sgd(true, X, k, l, p, V, ws, ws_bytes, stream);
}

int ppca_stream_pass(const ppca_matrix* X, int32_t K, const float* V, int64_t r0, int64_t nrows,
                     float* Z, double* G, void* ws, size_t ws_bytes, void* stream) {
  RET_IF(check_matrix(X));
  if (!V || !Z || r0 < 0 || r0 >= X->n || nrows < 1) return PPCA_ERR_ARG;
  RET_IF(check_k(X, K));
  const Plan p = make_plan(PPCA_OP_STREAM, X->n, X->d, X->dtype, K, nrows);
  RET_IF(check_ws(ws, ws_bytes, p));
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_zero(at<int>(ws, p.status), 256, s));
  RET_IF(make_operand(X, V, p, ws, s));
  RET_IF(run_pass(X, p, ws, r0, nrows, Z, G, nullptr, false, s));
  return finish(p, ws, s);
}

int ppca_project_gram(const ppca_matrix* X, int32_t K, const float* V, double* G, double* B,
                      void* ws, size_t ws_bytes, void* stream) {
  RET_IF(check_matrix(X));
  if (!V || !G || !B) return PPCA_ERR_ARG;
  RET_IF(check_k(X, K));
  const Plan p = make_plan(PPCA_OP_PROJECT, X->n, X->d, X->dtype, K, 0);
  RET_IF(check_ws(ws, ws_bytes, p));
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_zero(at<int>(ws, p.status), 256, s));
  RET_IF(make_operand(X, V, p, ws, s));
  RET_IF(operand_gram(X, V, p, ws, B, s));
  RET_IF(run_pass(X, p, ws, 0, X->n, nullptr, G, nullptr, true, s));
  return finish(p, ws, s);
}

int ppca_project_gram_rows(const ppca_matrix* X, int32_t K, const float* V, int64_t r0,
                           int64_t nrows, double* G, double* B, void* ws, size_t ws_bytes,
                           void* stream) {
  RET_IF(check_matrix(X));
  if (!V || !G || !B || r0 < 0 || r0 >= X->n || nrows < 1) return PPCA_ERR_ARG;
  RET_IF(check_k(X, K));
  const Plan p = make_plan(PPCA_OP_PROJECT, X->n, X->d, X->dtype, K, nrows);
  RET_IF(check_ws(ws, ws_bytes, p));
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_zero(at<int>(ws, p.status), 256, s));
  RET_IF(make_operand(X, V, p, ws, s));
  RET_IF(operand_gram(X, V, p, ws, B, s));
  RET_IF(run_pass(X, p, ws, r0, nrows, nullptr, G, nullptr, true, s));
  return finish(p, ws, s);
}

int ppca_rayleigh_ritz(const ppca_matrix* X, int32_t K, int32_t k, const double* G,
                       const double* B, const float* V, float* E, double* evals, void* ws,
                       size_t ws_bytes, void* stream) {
  RET_IF(check_rr(X, K, k, G, B, V, E, evals));
  const Plan p = make_plan(PPCA_OP_RR, X->n, X->d, X->dtype, K, 0);
  RET_IF(check_ws(ws, ws_bytes, p));
  return rayleigh_ritz_on(X, K, k, G, B, V, E, evals, p, ws, (hipStream_t)stream);
}

int ppca_rayleigh_ritz_noalloc(const ppca_matrix* X, int32_t K, int32_t k, const double* G,
                               const double* B, const float* V, float* E, double* evals,
                               void* stream) {
  RET_IF(check_rr(X, K, k, G, B, V, E, evals));
  const Plan p = make_plan(PPCA_OP_RR, X->n, X->d, X->dtype, K, 0);
  if (p.total > kStaticScratchBytes) return PPCA_ERR_WORKSPACE;
  void* ws = nullptr;
  RET_IF(static_scratch((hipStream_t)stream, &ws));
  return rayleigh_ritz_on(X, K, k, G, B, V, E, evals, p, ws, (hipStream_t)stream);
}

int ppca_prime_power_grouped(const ppca_problem* probs, int32_t nprob, int32_t iters,
                             int32_t flags, void* ws, size_t ws_bytes, void* stream) {
  if (iters < 0 || (flags & ~PPCA_GROUP_GRAPH) != 0) return PPCA_ERR_ARG;
  if (!probs || nprob < 1) return PPCA_ERR_ARG;
  for (int p = 0; p < nprob; ++p)
    if (!probs[p].V || !probs[p].G || !probs[p].B) return PPCA_ERR_ARG;
  GroupPlan gp;
  RET_IF(make_group_plan(probs, nprob, gp));
  RET_IF(check_group_ws(ws, ws_bytes, gp));
  hipStream_t s = (hipStream_t)stream;
  const bool graph = (flags & PPCA_GROUP_GRAPH) != 0;
  if (graph && s == nullptr) return PPCA_ERR_ARG;
  bind_group_plan(gp, probs, ws);
  RET_IF(upload_group_plan(gp, ws, s));
  const GProb* dP = at<GProb>(ws, gp.probs);
  int* st = at<int>(ws, gp.status);
  HIP_TRY(launch_group_cholqr2(dP, at<int>(ws, gp.order), nprob, true, iters == 0, st, s));
  if (graph && iters > 1) {
    // iterations 1 .. iters-1 replay one captured iteration; the last one
    // (which also forms B) runs eagerly
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const int rc = group_iteration(gp, ws, false, false, s);
    const hipError_t ec = hipStreamEndCapture(s, &g);
    if (rc != PPCA_OK || ec != hipSuccess) {
      if (g) hipGraphDestroy(g);
      return rc != PPCA_OK ? rc : PPCA_ERR_HIP;
    }
    const hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (ei != hipSuccess) return PPCA_ERR_HIP;
    hipError_t el = hipSuccess;
    for (int t = 0; t + 1 < iters && el == hipSuccess; ++t) el = hipGraphLaunch(ge, s);
    const hipError_t es = hipStreamSynchronize(s);
    hipGraphExecDestroy(ge);
    if (el != hipSuccess || es != hipSuccess) return PPCA_ERR_HIP;
    RET_IF(group_iteration(gp, ws, true, false, s));
  } else {
    for (int t = 0; t < iters; ++t) RET_IF(group_iteration(gp, ws, t == iters - 1, !graph, s));
  }
  // projection pass on the primed directions: G only
  const int nitems = (int)gp.hi.size();
  auto pass = [&] {
    return launch_group_pass(dP, at<GItem>(ws, gp.items), nitems, std::min(nitems, kNumCU),
                             at<float>(ws, gp.zpart), at<float>(ws, gp.gpart), false, s);
  };
  HIP_TRY(graph ? pass() : timed(2, s, pass));
  HIP_TRY(launch_group_reduce(dP, nprob, at<int>(ws, gp.blk_g), gp.bg.back(),
                              at<float>(ws, gp.zpart), at<float>(ws, gp.gpart), false, st, s));
  return finish_group(gp, ws, s);
}

int ppca_rayleigh_ritz_grouped(const ppca_problem* probs, int32_t nprob, void* ws,
                               size_t ws_bytes, void* stream) {
  if (!probs || nprob < 1) return PPCA_ERR_ARG;
  for (int p = 0; p < nprob; ++p)
    if (!probs[p].G || !probs[p].B || !probs[p].evals || !probs[p].V) return PPCA_ERR_ARG;
  GroupPlan gp;
  RET_IF(make_group_plan(probs, nprob, gp));
  RET_IF(check_group_ws(ws, ws_bytes, gp));
  hipStream_t s = (hipStream_t)stream;
  bind_group_plan(gp, probs, ws);
  RET_IF(upload_group_plan(gp, ws, s));
  HIP_TRY(launch_group_rr(at<GProb>(ws, gp.probs), at<int>(ws, gp.order), nprob, 60,
                          at<int>(ws, gp.status), s));
  return finish_group(gp, ws, s);
}

size_t ppca_grouped_workspace_bytes(const ppca_problem* probs, int32_t nprob) {
  GroupPlan gp;
  if (make_group_plan(probs, nprob, gp) != PPCA_OK) return 0;
  return gp.total;
}

size_t ppca_grouped_workspace_bytes_for(const ppca_problem* probs, int32_t nprob,
                                        int64_t item_bytes) {
  if (item_bytes < kGroupItemMin || item_bytes > kGroupItemMax) return 0;
  GroupPlan gp;
  if (make_group_plan(probs, nprob, gp, item_bytes) != PPCA_OK) return 0;
  return gp.total;
}

int ppca_set_group_item_bytes(int64_t bytes) {
  if (bytes == 0) bytes = kGroupItemBytes;
  if (bytes < kGroupItemMin || bytes > kGroupItemMax) return PPCA_ERR_ARG;
  g_group_item_bytes.store(bytes);
  return PPCA_OK;
}

int ppca_tune_group_items(const ppca_problem* probs, int32_t nprob, const int64_t* cand,
                          int32_t ncand, void* ws, size_t ws_bytes, void* stream,
                          int64_t* best_bytes, double* times_ms) {
  static const int64_t kDefault[] = {1 << 20, 2 << 20, 3 << 20, 4 << 20, 6 << 20, 8 << 20};
  if (!cand || ncand == 0) {
    cand = kDefault;
    ncand = (int32_t)(sizeof(kDefault) / sizeof(kDefault[0]));
  }
  if (ncand < 0 || !best_bytes || !probs || nprob < 1) return PPCA_ERR_ARG;
  for (int i = 0; i < ncand; ++i)
    if (cand[i] < kGroupItemMin || cand[i] > kGroupItemMax) return PPCA_ERR_ARG;
  for (int p = 0; p < nprob; ++p)
    if (!probs[p].V) return PPCA_ERR_ARG;
  // every candidate's plan must fit before anything runs
  for (int i = 0; i < ncand; ++i) {
    GroupPlan gp;
    RET_IF(make_group_plan(probs, nprob, gp, cand[i]));
    RET_IF(check_group_ws(ws, ws_bytes, gp));
  }
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    return PPCA_ERR_HIP;
  }
  int rc = PPCA_OK;
  double best = 0.0;
  for (int i = 0; i < ncand && rc == PPCA_OK; ++i) {
    GroupPlan gp;
    rc = make_group_plan(probs, nprob, gp, cand[i]);
    if (rc != PPCA_OK) break;
    bind_group_plan(gp, probs, ws);
    rc = upload_group_plan(gp, ws, s);
    if (rc != PPCA_OK) break;
    const GProb* dP = at<GProb>(ws, gp.probs);
    const int nitems = (int)gp.hi.size();
    auto pass = [&] {
      return launch_group_pass(dP, at<GItem>(ws, gp.items), nitems, std::min(nitems, kNumCU),
                               at<float>(ws, gp.zpart), at<float>(ws, gp.gpart), true, s);
    };
    // the operand of V as it stands, one untimed pass, then the timed one
    if (launch_group_operand(dP, nprob, s) != hipSuccess || pass() != hipSuccess ||
        hipEventRecord(e0, s) != hipSuccess || pass() != hipSuccess ||
        hipEventRecord(e1, s) != hipSuccess) {
      rc = PPCA_ERR_HIP;
      break;
    }
    rc = finish_group(gp, ws, s);   // synchronises: the host tables outlive their copies
    if (rc != PPCA_OK) break;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = PPCA_ERR_HIP;
      break;
    }
    if (times_ms) times_ms[i] = ms;
    if (i == 0 || ms < best) {
      best = ms;
      *best_bytes = cand[i];
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return rc;
}

size_t ppca_workspace_bytes(int32_t op, const ppca_matrix* X, int32_t K, int32_t batch) {
  if (!X || X->n < 1 || X->d < 1) return 0;
  if (op < PPCA_OP_CENTER || op > PPCA_OP_POWER_SEQ) return 0;
  if (op != PPCA_OP_CENTER && (K < 1 || K > PPCA_MAX_K)) return 0;
  if ((op == PPCA_OP_OJA || op == PPCA_OP_EIGENGAME) && (batch < 1 || batch > X->n)) return 0;
  if (op == PPCA_OP_STREAM && batch < 1) return 0;
  if (op == PPCA_OP_PROJECT && (batch < 0 || batch > X->n)) return 0;
  if (op == PPCA_OP_POWER_SEQ) return make_seq_plan(X->n, X->d, X->dtype).total;
  const Plan p = make_plan(op, X->n, X->d, X->dtype, op == PPCA_OP_CENTER ? 1 : K, batch);
  return p.total;
}

const char* ppca_strerror(int status) {
  switch (status) {
    case PPCA_OK: return "success";
    case PPCA_ERR_ARG: return "invalid argument";
    case PPCA_ERR_DTYPE: return "invalid dtype or col_scale";
    case PPCA_ERR_NOT_SPD: return "Cholesky pivot not positive: directions are rank deficient";
    case PPCA_ERR_NONFINITE: return "non-finite value in Z or a Gram matrix";
    case PPCA_ERR_NO_CONVERGENCE: return "Jacobi eigensolver reached its sweep cap";
    case PPCA_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case PPCA_ERR_HIP: return "HIP runtime error";
    case PPCA_ERR_ALIGN: return "X base pointer or row stride not 16-byte aligned";
    case PPCA_ERR_PLACEMENT: return "single-read pass: workgroups of a cluster not on one XCD";
    case PPCA_ERR_TIMEOUT: return "single-read pass: a bounded wait between workgroups expired";
    default: return "unknown status";
  }
}

void ppca_set_kernel_timing(int32_t enable) {
  std::lock_guard<std::mutex> lk(g_tmu);
  g_timing = enable != 0;
  for (auto& st : g_stats) st = KStat();
}

int ppca_kernel_stats(int32_t kernel, int64_t* launches, double* total_ms) {
  if (kernel < 0 || kernel > 5) return PPCA_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_tmu);
  if (launches) *launches = g_stats[kernel].launches;
  if (total_ms) *total_ms = g_stats[kernel].ms;
  return PPCA_OK;
}

int ppca_read_probe(const ppca_matrix* X, int32_t mode, int32_t seg_bytes, uint32_t* sink,
                    int64_t sink_len, void* stream) {
  RET_IF(check_matrix(X));
  if (mode != 0 && mode != 1) return PPCA_ERR_ARG;
  if (mode == 1 && seg_bytes != 128 && seg_bytes != 256 && seg_bytes != 512) return PPCA_ERR_ARG;
  if (!sink || sink_len < probe_grid(mode)) return PPCA_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  const int64_t row_bytes = X->ld * elem_size(X->dtype);
  HIP_TRY(timed(5, s, [&] {
    return launch_read_probe(X->x, X->n, row_bytes, mode, seg_bytes, sink, s);
  }));
  if (hipStreamSynchronize(s) != hipSuccess) return PPCA_ERR_HIP;
  if (g_timing) resolve_timings();
  return PPCA_OK;
}

void ppca_set_chunk_rows(int64_t rows) { g_chunk_rows.store(rows < 0 ? 0 : rows); }

void ppca_set_fused_pass(int32_t enable) { g_fused_enabled.store(enable != 0 ? 1 : 0); }

}  // extern "C"
