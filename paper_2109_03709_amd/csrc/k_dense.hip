// Small dense float64 kernels around the streaming passes:
//   * the MFMA operand V' (its float64 values V_eff are recomputed from V
//     where needed: the operand Gram B and the Ritz rotation),
//   * Gram matrices A^T A of tall d x K blocks (CholeskyQR2, B = V'^T V'),
//   * Cholesky with an explicit inverse of the triangular factor,
//   * Q = A R^-1 (CholeskyQR2), small K x K products (Rayleigh-Ritz),
//   * a parallel (round-robin) two-sided Jacobi eigensolver for K <= 128,
//   * the Ritz-vector rotation E = V_eff M and the output sign rule.
// Every reduction runs in a fixed order, so results are bitwise reproducible.
#include "dense_dev.h"

namespace ppca {

namespace {

using dev::kEps;
using dev::status_set;
constexpr int kJacRows = dev::kJacRows;

// --------------------------------------------------------------------------
// Operand: vop[c][j] (c < Kp, j < dp; zero outside d x K), and for the
// two-term operand the low terms at vop[Kp dp + c dp + j].  One workgroup
// transposes a 256-row x 16-column tile of V through LDS, so that both the
// reads of V (row-major) and the writes of vop (column-major) are coalesced.
// The float64 value an operand entry stands for is recomputed where it is
// needed (operand_value), never stored: at d in the millions it would be the
// largest buffer after X.
// --------------------------------------------------------------------------
constexpr int kOpRows = 256;   // rows of V per tile
constexpr int kOpCols = 16;    // columns per tile (Kp is a multiple of 16)

__global__ __launch_bounds__(256) void k_make_operand(const float* __restrict__ V, int64_t d, int K,
                                                      int64_t dp, int dtype,
                                                      const float* __restrict__ scale,
                                                      void* __restrict__ vop, int64_t total,
                                                      int split) {
  __shared__ float tile[kOpCols][kOpRows + 1];
  const int t = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * kOpRows;
  const int c0 = (int)blockIdx.y * kOpCols;
#pragma unroll
  for (int q = 0; q < kOpRows * kOpCols / 256; ++q) {
    const int i = t + 256 * q;
    const int r = i / kOpCols, cc = i % kOpCols;
    const int64_t j = j0 + r;
    const int c = c0 + cc;
    tile[cc][r] = (j < d && c < K) ? V[j * K + c] : 0.f;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kOpRows * kOpCols / 256; ++q) {
    const int i = t + 256 * q;
    const int cc = i / kOpRows, r = i % kOpRows;
    const int64_t j = j0 + r;
    if (j >= dp) continue;
    const int64_t e = (int64_t)(c0 + cc) * dp + j;
    const float v = tile[cc][r];
    if (dtype == PPCA_F32) {
      reinterpret_cast<float*>(vop)[e] = v;
    } else {
      const float sv = (dtype == PPCA_FP8_E4M3 && j < d) ? scale[j] * v : v;
      const uint32_t h = f32_to_bf16_bits(sv);
      reinterpret_cast<uint16_t*>(vop)[e] = (uint16_t)h;
      if (split) {
        // sv - hi has at most 16 significant bits: exact in float32
        const uint32_t lo = f32_to_bf16_bits(sv - bf16_bits_to_f32(h));
        reinterpret_cast<uint16_t*>(vop)[total + e] = (uint16_t)lo;
      }
    }
  }
}

// The float64 value the operand holds for entry v of row j (j < d): v itself
// for float32 data; else the bf16 rounding of v (of scale_j v for fp8 data,
// divided back by scale_j), plus the bf16 rounding of the remainder for the
// two-term operand.  Same arithmetic as k_make_operand, entry by entry.
__device__ inline double operand_value(float v, int64_t j, int dtype, int split,
                                       const float* __restrict__ scale) {
  if (dtype == PPCA_F32) return (double)v;
  const float sv = dtype == PPCA_FP8_E4M3 ? scale[j] * v : v;
  const uint32_t h = f32_to_bf16_bits(sv);
  double ve = (double)bf16_bits_to_f32(h);
  if (split) ve += (double)bf16_bits_to_f32(f32_to_bf16_bits(sv - bf16_bits_to_f32(h)));
  if (dtype == PPCA_FP8_E4M3) ve = ve / (double)scale[j];
  return ve;
}

// --------------------------------------------------------------------------
// Gram partials of a (rows x K) matrix A: block (tile pair, chunk) computes the
// 32 x 32 tile (ti, tj), ti <= tj, of A[rows of chunk]^T A[rows of chunk] in
// float64; parts[chunk] holds the upper tiles.  k_sum_gram adds the chunks in
// order and mirrors the lower tiles.
// --------------------------------------------------------------------------
constexpr int kGT = 32;            // Gram output tile
constexpr int kGR = 64;            // rows staged per step

// OPV: A is V (float32, lda = K) and the Gram is taken of the operand values
// operand_value(V[row][c], row, dtype, split, scale).
template <typename T, bool OPV = false>
__global__ __launch_bounds__(256) void k_gram_tile(const T* __restrict__ A, int64_t rows, int K,
                                                   int64_t lda, int nchunk,
                                                   double* __restrict__ parts, int dtype = 0,
                                                   int split = 0,
                                                   const float* __restrict__ scale = nullptr) {
  __shared__ double Ai[kGR][kGT + 1], Aj[kGR][kGT + 1];
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  const int nt = (K + kGT - 1) / kGT;
  int pidx = blockIdx.x, ti = 0;
  while (pidx >= nt - ti) {
    pidx -= nt - ti;
    ++ti;
  }
  const int tj = ti + pidx;
  const int64_t rpc = (rows + nchunk - 1) / nchunk;
  const int64_t rb = (int64_t)blockIdx.y * rpc;
  const int64_t re = rb + rpc < rows ? rb + rpc : rows;
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int64_t r0 = rb; r0 < re; r0 += kGR) {
#pragma unroll
    for (int e = t; e < kGR * kGT; e += 256) {   // fixed trip count: all loads issued first
      const int r = e / kGT, c = e % kGT;
      const int64_t row = r0 + r;
      const int ci = ti * kGT + c, cj = tj * kGT + c;
      if constexpr (OPV) {
        Ai[r][c] = (row < re && ci < K) ? operand_value(A[row * lda + ci], row, dtype, split, scale)
                                        : 0.0;
        Aj[r][c] = (row < re && cj < K) ? operand_value(A[row * lda + cj], row, dtype, split, scale)
                                        : 0.0;
      } else {
        Ai[r][c] = (row < re && ci < K) ? (double)A[row * lda + ci] : 0.0;
        Aj[r][c] = (row < re && cj < K) ? (double)A[row * lda + cj] : 0.0;
      }
    }
    __syncthreads();
    const int nr = (int)(re - r0 < kGR ? re - r0 : kGR);
    for (int r = 0; r < nr; ++r) {
      const double a0 = Ai[r][2 * ty], a1 = Ai[r][2 * ty + 1];
      const double b0 = Aj[r][2 * tx], b1 = Aj[r][2 * tx + 1];
      acc[0][0] = fma(a0, b0, acc[0][0]);
      acc[0][1] = fma(a0, b1, acc[0][1]);
      acc[1][0] = fma(a1, b0, acc[1][0]);
      acc[1][1] = fma(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
  double* out = parts + (int64_t)blockIdx.y * K * K;
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int i = ti * kGT + 2 * ty + u, j = tj * kGT + 2 * tx + v;
      if (i < K && j < K) out[i * K + j] = acc[u][v];
    }
}

__global__ __launch_bounds__(256) void k_sum_gram(const double* __restrict__ parts, int nparts,
                                                  int K, double* __restrict__ out, int* status) {
  bool bad = false;
  const int64_t count = (int64_t)K * K;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / K), j = (int)(e % K);
    const int64_t src = (i / kGT <= j / kGT) ? e : (int64_t)j * K + i;   // lower tiles: mirror
    // chunks in order, eight loads in flight at a time (the same sum as one
    // load per step, without a dependent L2 round trip per chunk)
    const double* q = parts + src;
    double sacc = 0.0;
    int p = 0;
    for (; p + 8 <= nparts; p += 8) {
      double v[8];
#pragma unroll
      for (int w = 0; w < 8; ++w) v[w] = q[(int64_t)(p + w) * count];
#pragma unroll
      for (int w = 0; w < 8; ++w) sacc += v[w];
    }
    for (; p < nparts; ++p) sacc += q[(int64_t)p * count];
    if (!isfinite(sacc)) bad = true;
    out[e] = sacc;
  }
  if (bad) set_status(status, PPCA_ERR_NONFINITE);
}

// Cholesky factor and inverse of one K x K matrix (body in dense_dev.h).
__global__ __launch_bounds__(256) void k_chol_inv(const double* __restrict__ A, int K,
                                                   double* __restrict__ R,
                                                   double* __restrict__ Rinv, int* status) {
  __shared__ double lds[dev::chol_lds_doubles<kMaxK>()];
  dev::chol_inv_dev<kMaxK>(A, K, R, Rinv, status, lds);
}

// --------------------------------------------------------------------------
// out = A * Rinv for upper-triangular Rinv (K x K): tiled product, block =
// 64 rows x 32 columns of out.  Rinv is zero below its diagonal, so the
// block needs the columns [0, kend) of its rows of A and the rows [0, kend)
// of its columns of Rinv, kend = min(c0 + 32, K): all of them are loaded in
// one batch (every load in flight before the first is used), staged in LDS,
// and the k loop runs over them in order.
// --------------------------------------------------------------------------
constexpr int kTR = 64, kTC = 32;

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_trmm(const TI* __restrict__ A, int64_t rows, int K,
                                              int64_t lda, const double* __restrict__ Rinv,
                                              TO* __restrict__ out, int64_t ldo, int* status) {
  __shared__ double As[kTR][kMaxK + 1], Rs[kMaxK][kTC + 1];
  if (status_set(status)) return;
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * kTR;
  const int c0 = blockIdx.y * kTC;
  const int kend = c0 + kTC < K ? c0 + kTC : K;
  constexpr int NA = kTR * kMaxK / 256, NR = kMaxK * kTC / 256;
  double va[NA], vr[NR];
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    const int e = t + 256 * u, r = e / kMaxK, c = e % kMaxK;
    const int64_t row = r0 + r;
    va[u] = (row < rows && c < kend) ? (double)A[row * lda + c] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < NR; ++u) {
    const int e = t + 256 * u, r = e / kTC, c = e % kTC;
    vr[u] = (r < kend && c0 + c < K) ? Rinv[r * K + c0 + c] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    const int e = t + 256 * u;
    As[e / kMaxK][e % kMaxK] = va[u];
  }
#pragma unroll
  for (int u = 0; u < NR; ++u) {
    const int e = t + 256 * u;
    Rs[e / kTC][e % kTC] = vr[u];
  }
  __syncthreads();
  double acc[4][2] = {};
  for (int pp = 0; pp < kend; ++pp) {
    const double b0 = Rs[pp][2 * tx], b1 = Rs[pp][2 * tx + 1];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double av = As[4 * ty + u][pp];
      acc[u][0] = fma(av, b0, acc[u][0]);
      acc[u][1] = fma(av, b1, acc[u][1]);
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t row = r0 + 4 * ty + u;
    if (row >= rows) continue;
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int col = c0 + 2 * tx + v;
      if (col < K) out[row * ldo + col] = (TO)acc[u][v];
    }
  }
}

// --------------------------------------------------------------------------
// C[M][N] = alpha * op(A) * B, op(A) = A (M x Kd) or A^T (A is Kd x M).
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_small_gemm(const double* __restrict__ A, int transA,
                                                    const double* __restrict__ B,
                                                    double* __restrict__ C, int M, int N, int Kd,
                                                    int lda, int ldb, int ldc, double alpha,
                                                    int* status) {
  if (status_set(status)) return;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < M * N; e += gridDim.x * blockDim.x) {
    const int i = e / N, j = e % N;
    double s = 0.0;
    for (int p = 0; p < Kd; ++p) {
      const double av = transA ? A[p * lda + i] : A[i * lda + p];
      s = fma(av, B[p * ldb + j], s);
    }
    C[i * ldc + j] = alpha * s;
  }
}

// Jacobi eigensolver, one 16-row block of W per workgroup (body in dense_dev.h).
__global__ __launch_bounds__(1024) void k_jacobi(const double* __restrict__ H, int K,
                                                 double* __restrict__ Ws, double* __restrict__ evals,
                                                 int max_sweeps, int* status) {
  dev::jacobi_dev<kMaxK>(H, K, Ws, evals, max_sweeps, status, blockIdx.x);
}

// --------------------------------------------------------------------------
// Ritz vectors E[j][c] = sum_p veff[j][p] M[p][c] (float64 accumulate, float32
// out), veff the operand values of V, then the sign rule: column c is negated
// when its largest-|.| entry (lowest row on ties) is negative.
//   k_rotate      E, and per workgroup and column the largest |E| entry
//                 (value and row) among the rows the workgroup wrote;
//   k_sign_decide one workgroup: per column the largest entry over the
//                 workgroups (the same entry whatever the order), its sign;
//   k_flip        negates the flagged columns.
// A tile is R = 1024 / k rows of E (R k <= 1024 entries, four per thread);
// thread t always holds tile entries t + 256 q, so its columns are fixed and
// it keeps a running maximum for each.
// --------------------------------------------------------------------------
constexpr int kRotTile = 1024;
constexpr int kRotMaxBlocks = 1024;

__device__ inline bool colmax_better(float a, int64_t j, float ba, int64_t bj) {
  return a > ba || (a == ba && j < bj);
}

// MS: LDS entries for M (K k <= MS).
template <int MS>
__global__ __launch_bounds__(256) void k_rotate(const float* __restrict__ V, int64_t d, int K,
                                                int dtype, int split,
                                                const float* __restrict__ scale,
                                                const double* __restrict__ M, int k,
                                                float* __restrict__ E, ColMax* __restrict__ part,
                                                int* status) {
  __shared__ double Ms[MS];
  __shared__ ColMax sm[kRotTile];
  if (status_set(status)) return;
  for (int e = threadIdx.x; e < K * k; e += blockDim.x) Ms[e] = M[e];
  __syncthreads();
  const int R = kRotTile / k > 0 ? kRotTile / k : 1;
  const int nel = R * k;
  const int64_t ntiles = (d + R - 1) / R;
  float ba[4], bv[4];
  int64_t bj[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    ba[q] = -1.f;
    bv[q] = 0.f;
    bj[q] = INT64_MAX;
  }
  for (int64_t tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = threadIdx.x + 256 * q;
      if (i >= nel) continue;
      const int64_t j = tl * R + i / k;
      const int c = i % k;
      if (j >= d) continue;
      const float* vr = V + j * K;
      double s = 0.0;
      for (int p = 0; p < K; ++p) s = fma(operand_value(vr[p], j, dtype, split, scale), Ms[p * k + c], s);
      const float ef = (float)s;
      E[j * k + c] = ef;
      const float a = fabsf(ef);
      if (colmax_better(a, j, ba[q], bj[q])) {
        ba[q] = a;
        bv[q] = ef;
        bj[q] = j;
      }
    }
  }
  // the block's maximum per column over its threads' slots
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = threadIdx.x + 256 * q;
    if (i < nel) sm[i] = ColMax{ba[q], bv[q], bj[q]};
  }
  __syncthreads();
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    ColMax b{-1.f, 0.f, INT64_MAX};
    for (int i = c; i < nel; i += k)
      if (colmax_better(sm[i].a, sm[i].j, b.a, b.j)) b = sm[i];
    part[(int64_t)blockIdx.x * k + c] = b;
  }
}

__global__ __launch_bounds__(256) void k_sign_decide(const ColMax* __restrict__ part, int nblk,
                                                     int k, int* __restrict__ flip, int* status) {
  if (status_set(status)) return;
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    ColMax b{-1.f, 0.f, INT64_MAX};
    for (int w = 0; w < nblk; ++w) {
      const ColMax m = part[(int64_t)w * k + c];
      if (colmax_better(m.a, m.j, b.a, b.j)) b = m;
    }
    flip[c] = b.a >= 0.f && b.v < 0.f;
  }
}

__global__ __launch_bounds__(256) void k_flip(float* __restrict__ E, int64_t d, int k,
                                              const int* __restrict__ flip, int* status) {
  if (status_set(status)) return;
  const int R = kRotTile / k > 0 ? kRotTile / k : 1;
  const int nel = R * k;
  const int64_t ntiles = (d + R - 1) / R;
  for (int64_t tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = threadIdx.x + 256 * q;
      if (i >= nel) continue;
      const int64_t j = tl * R + i / k;
      const int c = i % k;
      if (j < d && flip[c]) E[j * k + c] = -E[j * k + c];
    }
  }
}

__global__ void k_copy_f64(const double* __restrict__ s, double* __restrict__ d, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    d[e] = s[e];
}

__global__ void k_zero(uint32_t* __restrict__ p, int64_t words) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < words;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = 0u;
}

inline int64_t grid_for(int64_t n, int64_t cap = 4096) {
  int64_t g = cdiv(n, 256);
  if (g < 1) g = 1;
  return g > cap ? cap : g;
}

}  // namespace

hipError_t launch_make_operand(const float* V, int64_t d, int K, int Kp, int64_t dp, int32_t dtype,
                               const float* col_scale, void* vop, bool split, hipStream_t s) {
  if (Kp % kOpCols != 0) return hipErrorInvalidValue;
  const dim3 grid((unsigned)cdiv(dp, kOpRows), (unsigned)(Kp / kOpCols));
  hipLaunchKernelGGL(k_make_operand, grid, dim3(256), 0, s, V, d, K, dp, (int)dtype, col_scale,
                     vop, (int64_t)Kp * dp, split ? 1 : 0);
  return hipGetLastError();
}

static int gram_tiles(int K) {
  const int nt = (int)cdiv(K, kGT);
  return nt * (nt + 1) / 2;
}

// row chunks of the Gram: about 512 blocks in all, at least 128 rows a chunk
// (at d = 2048, K = 128: 16 chunks of two 64-row stages; the fixed-order sum
// over the chunks then reads 16 partials instead of 52)
int gram_parts(int64_t rows, int K) {
  int64_t nc = cdiv(512, gram_tiles(K));
  const int64_t by_rows = cdiv(rows, 128);
  if (nc > by_rows) nc = by_rows;
  if (nc < 1) nc = 1;
  return (int)nc;
}

hipError_t launch_gram(const void* A, bool in_f64, int64_t rows, int K, int64_t lda, double* parts,
                       double* out, int* status, hipStream_t s) {
  const int np = gram_parts(rows, K);
  const dim3 grid(gram_tiles(K), np);
  if (in_f64)
    hipLaunchKernelGGL(k_gram_tile<double>, grid, dim3(256), 0, s, (const double*)A, rows, K, lda,
                       np, parts);
  else
    hipLaunchKernelGGL(k_gram_tile<float>, grid, dim3(256), 0, s, (const float*)A, rows, K, lda,
                       np, parts);
  hipLaunchKernelGGL(k_sum_gram, dim3(grid_for((int64_t)K * K)), dim3(256), 0, s, parts, np, K,
                     out, status);
  return hipGetLastError();
}

hipError_t launch_operand_gram(const float* V, int64_t d, int K, int32_t dtype, bool split,
                               const float* col_scale, double* parts, double* out, int* status,
                               hipStream_t s) {
  const int np = gram_parts(d, K);
  const dim3 grid(gram_tiles(K), np);
  hipLaunchKernelGGL((k_gram_tile<float, true>), grid, dim3(256), 0, s, V, d, K, (int64_t)K, np,
                     parts, (int)dtype, split ? 1 : 0, col_scale);
  hipLaunchKernelGGL(k_sum_gram, dim3(grid_for((int64_t)K * K)), dim3(256), 0, s, parts, np, K,
                     out, status);
  return hipGetLastError();
}

hipError_t launch_chol_inv(const double* A, int K, double* R, double* Rinv, int* status,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(256), 0, s, A, K, R, Rinv, status);
  return hipGetLastError();
}

hipError_t launch_trmm(const void* A, bool in_f64, int64_t rows, int K, int64_t lda,
                       const double* Rinv, void* out, bool out_f64, int64_t ldo, int* status,
                       hipStream_t s) {
  const dim3 grid((unsigned)cdiv(rows, kTR), (unsigned)cdiv(K, kTC));
  if (in_f64 && out_f64)
    hipLaunchKernelGGL((k_trmm<double, double>), grid, dim3(256), 0, s, (const double*)A, rows, K,
                       lda, Rinv, (double*)out, ldo, status);
  else if (in_f64)
    hipLaunchKernelGGL((k_trmm<double, float>), grid, dim3(256), 0, s, (const double*)A, rows, K,
                       lda, Rinv, (float*)out, ldo, status);
  else if (out_f64)
    hipLaunchKernelGGL((k_trmm<float, double>), grid, dim3(256), 0, s, (const float*)A, rows, K,
                       lda, Rinv, (double*)out, ldo, status);
  else
    hipLaunchKernelGGL((k_trmm<float, float>), grid, dim3(256), 0, s, (const float*)A, rows, K,
                       lda, Rinv, (float*)out, ldo, status);
  return hipGetLastError();
}

hipError_t launch_small_gemm(const double* A, bool transA, const double* B, double* C, int M,
                             int N, int Kd, int lda, int ldb, int ldc, double alpha, int* status,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_small_gemm, dim3(grid_for((int64_t)M * N, 256)), dim3(256), 0, s, A,
                     transA ? 1 : 0, B, C, M, N, Kd, lda, ldb, ldc, alpha, status);
  return hipGetLastError();
}

hipError_t launch_jacobi(const double* H, int K, double* W, double* evals, int max_sweeps,
                         int* status, hipStream_t s) {
  const int nwg = (int)cdiv(K, kJacRows);
  hipLaunchKernelGGL(k_jacobi, dim3(nwg), dim3(1024), 0, s, H, K, W, evals, max_sweeps, status);
  return hipGetLastError();
}

int rotate_blocks(int64_t d, int k) {
  const int64_t R = kRotTile / k > 0 ? kRotTile / k : 1;
  const int64_t nb = cdiv(d, R);
  return (int)(nb < kRotMaxBlocks ? nb : kRotMaxBlocks);
}

hipError_t launch_rotate(const float* V, int64_t d, int K, int32_t dtype, bool split,
                         const float* col_scale, const double* M, int k, float* E, ColMax* part,
                         int* flip, int* status, hipStream_t s) {
  if (k < 1 || k > K || K > kMaxK) return hipErrorInvalidValue;
  const int nb = rotate_blocks(d, k);
  if (K * k <= 1024)
    hipLaunchKernelGGL(k_rotate<1024>, dim3(nb), dim3(256), 0, s, V, d, K, (int)dtype,
                       split ? 1 : 0, col_scale, M, k, E, part, status);
  else
    hipLaunchKernelGGL(k_rotate<kMaxK * kMaxK>, dim3(nb), dim3(256), 0, s, V, d, K, (int)dtype,
                       split ? 1 : 0, col_scale, M, k, E, part, status);
  hipLaunchKernelGGL(k_sign_decide, dim3(1), dim3(256), 0, s, part, nb, k, flip, status);
  hipLaunchKernelGGL(k_flip, dim3(nb), dim3(256), 0, s, E, d, k, flip, status);
  return hipGetLastError();
}

hipError_t launch_copy_f64(const double* src, double* dst, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_f64, dim3(grid_for(count)), dim3(256), 0, s, src, dst, count);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  const int64_t words = (int64_t)(bytes / 4);
  hipLaunchKernelGGL(k_zero, dim3(grid_for(words)), dim3(256), 0, s, (uint32_t*)p, words);
  return hipGetLastError();
}

}  // namespace ppca
