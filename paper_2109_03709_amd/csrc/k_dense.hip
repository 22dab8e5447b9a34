// Small dense float64 kernels around the streaming passes:
//   * the MFMA operand V' and its float64 image V_eff (operand-exact basis),
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
// Operand: vop[c][j] (c < Kp, j < dp; zero outside d x K) and veff[j][c]
// (j < d, c < Kp; zero for c >= K).
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_make_operand(const float* __restrict__ V, int64_t d, int K,
                                                      int Kp, int64_t dp, int dtype,
                                                      const float* __restrict__ scale,
                                                      void* __restrict__ vop,
                                                      double* __restrict__ veff, int split) {
  const int64_t total = (int64_t)Kp * dp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / dp);
    const int64_t j = e % dp;
    const bool in = (j < d) && (c < K);
    const float v = in ? V[j * K + c] : 0.f;
    double ve = 0.0;
    if (dtype == PPCA_F32) {
      reinterpret_cast<float*>(vop)[e] = v;
      ve = (double)v;
    } else {
      const float sv = (dtype == PPCA_FP8_E4M3 && in) ? scale[j] * v : v;
      const uint32_t h = f32_to_bf16_bits(sv);
      reinterpret_cast<uint16_t*>(vop)[e] = (uint16_t)h;
      ve = (double)bf16_bits_to_f32(h);
      if (split) {
        // sv - hi has at most 16 significant bits: exact in float32
        const uint32_t lo = f32_to_bf16_bits(sv - bf16_bits_to_f32(h));
        reinterpret_cast<uint16_t*>(vop)[total + e] = (uint16_t)lo;
        ve += (double)bf16_bits_to_f32(lo);
      }
      if (dtype == PPCA_FP8_E4M3 && in) ve = ve / (double)scale[j];
    }
    if (j < d) veff[j * Kp + c] = ve;
  }
}

// --------------------------------------------------------------------------
// Gram partials of a (rows x K) matrix A: block (tile pair, chunk) computes the
// 32 x 32 tile (ti, tj), ti <= tj, of A[rows of chunk]^T A[rows of chunk] in
// float64; parts[chunk] holds the upper tiles.  k_sum_gram adds the chunks in
// order and mirrors the lower tiles.
// --------------------------------------------------------------------------
constexpr int kGT = 32;            // Gram output tile
constexpr int kGR = 64;            // rows staged per step

template <typename T>
__global__ __launch_bounds__(256) void k_gram_tile(const T* __restrict__ A, int64_t rows, int K,
                                                   int64_t lda, int nchunk,
                                                   double* __restrict__ parts) {
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
      Ai[r][c] = (row < re && ci < K) ? (double)A[row * lda + ci] : 0.0;
      Aj[r][c] = (row < re && cj < K) ? (double)A[row * lda + cj] : 0.0;
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
// 64 rows x 32 columns of out, k-steps of 32 that stop at the tile's last
// column (Rinv is zero below its diagonal).
// --------------------------------------------------------------------------
constexpr int kTR = 64, kTC = 32;

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_trmm(const TI* __restrict__ A, int64_t rows, int K,
                                              int64_t lda, const double* __restrict__ Rinv,
                                              TO* __restrict__ out, int64_t ldo, int* status) {
  __shared__ double As[kTR][kTC + 1], Rs[kTC][kTC + 1];
  if (status_set(status)) return;
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * kTR;
  const int c0 = blockIdx.y * kTC;
  const int kend = c0 + kTC < K ? c0 + kTC : K;
  double acc[4][2] = {};
  for (int p0 = 0; p0 < kend; p0 += kTC) {
#pragma unroll
    for (int e = t; e < kTR * kTC; e += 256) {   // fixed trip count: all loads issued first
      const int r = e / kTC, c = e % kTC;
      const int64_t row = r0 + r;
      const int col = p0 + c;
      As[r][c] = (row < rows && col < K) ? (double)A[row * lda + col] : 0.0;
    }
#pragma unroll
    for (int e = t; e < kTC * kTC; e += 256) {
      const int r = e / kTC, c = e % kTC;
      const int pr = p0 + r, pc = c0 + c;
      Rs[r][c] = (pr < K && pc < K) ? Rinv[pr * K + pc] : 0.0;
    }
    __syncthreads();
    for (int pp = 0; pp < kTC; ++pp) {
      const double b0 = Rs[pp][2 * tx], b1 = Rs[pp][2 * tx + 1];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double av = As[4 * ty + u][pp];
        acc[u][0] = fma(av, b0, acc[u][0]);
        acc[u][1] = fma(av, b1, acc[u][1]);
      }
    }
    __syncthreads();
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
// E[j][c] = sum_p veff[j][p] M[p][c]  (float64 accumulate, float32 out)
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_rotate(const double* __restrict__ veff, int64_t d, int Kp,
                                                int K, const double* __restrict__ M, int k,
                                                float* __restrict__ E, int* status) {
  __shared__ double Ms[kMaxK * kMaxK];
  if (status_set(status)) return;
  for (int e = threadIdx.x; e < K * k; e += blockDim.x) Ms[e] = M[e];
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < d * k;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / k;
    const int c = (int)(e % k);
    double s = 0.0;
    for (int p = 0; p < K; ++p) s = fma(veff[j * Kp + p], Ms[p * k + c], s);
    E[e] = (float)s;
  }
}

// Flip column c of E so that its largest-|.| entry (lowest row on ties) is positive.
__global__ __launch_bounds__(256) void k_sign_fix(float* __restrict__ E, int64_t d, int k,
                                                  int* status) {
  __shared__ float bv[256];
  __shared__ int64_t bi[256];
  if (status_set(status)) return;
  const int c = blockIdx.x;
  float best = -1.f;
  int64_t bidx = 0;
  for (int64_t j = threadIdx.x; j < d; j += blockDim.x) {
    const float v = fabsf(E[j * k + c]);
    if (v > best) { best = v; bidx = j; }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bidx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      const float v2 = bv[threadIdx.x + o];
      const int64_t i2 = bi[threadIdx.x + o];
      if (v2 > bv[threadIdx.x] || (v2 == bv[threadIdx.x] && i2 < bi[threadIdx.x])) {
        bv[threadIdx.x] = v2;
        bi[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  // One thread reads the pivot and publishes the decision; every thread
  // waits for it before any row is negated (the pivot row belongs to one of
  // the threads, which would otherwise negate it before the others read it).
  __shared__ int flip;
  if (threadIdx.x == 0) flip = E[bi[0] * k + c] < 0.f;
  __syncthreads();
  if (flip)
    for (int64_t j = threadIdx.x; j < d; j += blockDim.x) E[j * k + c] = -E[j * k + c];
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
                               const float* col_scale, void* vop, double* veff, bool split,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_make_operand, dim3(grid_for((int64_t)Kp * dp)), dim3(256), 0, s, V, d, K,
                     Kp, dp, (int)dtype, col_scale, vop, veff, split ? 1 : 0);
  return hipGetLastError();
}

static int gram_tiles(int K) {
  const int nt = (int)cdiv(K, kGT);
  return nt * (nt + 1) / 2;
}

// row chunks of the Gram: about 512 blocks in all, at least 16 rows a chunk
int gram_parts(int64_t rows, int K) {
  int64_t nc = cdiv(512, gram_tiles(K));
  const int64_t by_rows = cdiv(rows, 16);
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

hipError_t launch_rotate(const double* veff, int64_t d, int Kp, int K, const double* M, int k,
                         float* E, int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_rotate, dim3(grid_for(d * k, 1024)), dim3(256), 0, s, veff, d, Kp, K, M, k,
                     E, status);
  return hipGetLastError();
}

hipError_t launch_sign_fix(float* E, int64_t d, int k, int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_sign_fix, dim3(k), dim3(256), 0, s, E, d, k, status);
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
