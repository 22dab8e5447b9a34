// Small dense float64 kernels around the streaming passes:
//   * the MFMA operand V' and its float64 image V_eff (operand-exact basis),
//   * Gram matrices A^T A of tall d x K blocks (CholeskyQR2, B = V'^T V'),
//   * Cholesky with an explicit inverse of the triangular factor,
//   * Q = A R^-1 (CholeskyQR2), small K x K products (Rayleigh-Ritz),
//   * a parallel (round-robin) two-sided Jacobi eigensolver for K <= 128,
//   * the Ritz-vector rotation E = V_eff M and the output sign rule.
// Every reduction runs in a fixed order, so results are bitwise reproducible.
#include "ppca_common.h"

namespace ppca {

namespace {

constexpr double kEps = 2.220446049250313e-16;

__device__ inline bool status_set(const int* status) {
  return *reinterpret_cast<const volatile int*>(status) != 0;
}

// --------------------------------------------------------------------------
// Operand: vop[c][j] (c < Kp, j < dp; zero outside d x K) and veff[j][c]
// (j < d, c < Kp; zero for c >= K).
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_make_operand(const float* __restrict__ V, int64_t d, int K,
                                                      int Kp, int64_t dp, int dtype,
                                                      const float* __restrict__ scale,
                                                      void* __restrict__ vop,
                                                      double* __restrict__ veff) {
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
    double sacc = 0.0;
    for (int p = 0; p < nparts; ++p) sacc += parts[(int64_t)p * count + src];
    if (!isfinite(sacc)) bad = true;
    out[e] = sacc;
  }
  if (bad) set_status(status, PPCA_ERR_NONFINITE);
}

// --------------------------------------------------------------------------
// Upper Cholesky factor R (R^T R = A) and X = R^-1, K <= 128, one workgroup of
// 256 threads (one wavefront per SIMD: the register file holds the unrolled
// block steps), blocked in 16 x 16 blocks (the matrix is padded with the
// identity to a multiple of 16; the padding factors to the identity).
//
// Factorisation, for each block row J (three barriers per block row):
//   (1) wavefront 0 factors the diagonal block in registers (lane c holds
//       column c; pivots and row entries are broadcast with readlane).  Pivot
//       test: finite, > K * eps * |a_jj| and > 0, else NOT_SPD;
//   (2) one thread per column c > J solves R_JJ^T R_Jc = M_Jc (forward
//       substitution) for the row panel;
//   (3) the rank-16 update M_ic -= R_Ji^T R_Jc of the trailing upper
//       triangle, 4 x 4 elements per thread.
// Inverse: the diagonal blocks are inverted in place, one wavefront each;
// then for each block row I from the bottom: T = R_I,>I X_>I (the rows of X
// below are final; a thread owns one column and 4 rows of T), then
// X_I,>I = -R_II^-1 T; two barriers per block row.  T is kept in the unused
// strict lower triangle of the matrix.
// --------------------------------------------------------------------------
__device__ inline double bcast_lane(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

__global__ __launch_bounds__(256) void k_chol_inv(const double* __restrict__ A, int K,
                                                   double* __restrict__ R,
                                                   double* __restrict__ Rinv, int* status) {
  constexpr int KM = kMaxK, LDM = KM + 1, BS = 16;   // row stride 129: column reads spread banks
  __shared__ double M[KM * LDM];
  __shared__ double dg[KM];
  __shared__ double rcp[KM];         // 1 / r_jj
  __shared__ int fail;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (status_set(status)) return;
  const int nbk = (K + BS - 1) / BS, Kp = nbk * BS;
  if (tid == 0) fail = 0;
  // load A in batches of 16 elements per thread, all loads in flight before
  // any is used (a plain loop waits for every load in turn)
  for (int e0 = tid; e0 < Kp * Kp; e0 += 16 * 256) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + 256 * u;
      const int i = e / Kp, c = e - i * Kp;
      v[u] = (e < Kp * Kp && i < K && c < K && c >= i) ? A[i * K + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + 256 * u;
      if (e >= Kp * Kp) continue;
      const int i = e / Kp, c = e - i * Kp;
      const double w = (i < K && c < K) ? v[u] : (i == c ? 1.0 : 0.0);
      M[i * LDM + c] = w;
      if (i == c) dg[i] = w;
    }
  }
  __syncthreads();
  for (int J = 0; J < nbk; ++J) {
    const int j0 = J * BS;
    // (1) diagonal block in registers of wavefront 0 (lanes 16..63 idle)
    if (wave == 0) {
      const int c = lane & (BS - 1);
      double col[BS];
#pragma unroll
      for (int i = 0; i < BS; ++i) col[i] = (i <= c) ? M[(j0 + i) * LDM + j0 + c] : 0.0;
      bool ok = true;
#pragma unroll
      for (int p = 0; p < BS; ++p) {
        const double piv = bcast_lane(col[p], p);
        const int jp = j0 + p;
        // uniform: every lane holds the same pivot; after a failure the
        // values are garbage and are not stored
        ok = ok && isfinite(piv) && piv > (double)K * kEps * fabs(dg[jp]) && piv > 0.0;
        // one reciprocal square root per pivot; the row is scaled by it
        // (shorter dependency chain than a square root and a division)
        const double rinv = rsqrt(fabs(piv));
        const double rpp = fabs(piv) * rinv;
        const double u = (c > p) ? col[p] * rinv : 0.0;   // R[p][c]
        col[p] = (c == p) ? rpp : ((c > p) ? u : col[p]);
        if (lane == 0) rcp[jp] = rinv;
#pragma unroll
        for (int i = p + 1; i < BS; ++i) {
          const double ui = bcast_lane(u, i);
          if (i <= c) col[i] = fma(-ui, u, col[i]);
        }
      }
      if (!ok) {
        if (lane == 0) fail = 1;
      } else if (lane < BS) {
#pragma unroll
        for (int i = 0; i < BS; ++i)
          if (i <= c) M[(j0 + i) * LDM + j0 + c] = col[i];
      }
    }
    __syncthreads();
    if (fail) {
      if (tid == 0) set_status(status, PPCA_ERR_NOT_SPD);
      return;
    }
    const int n0 = j0 + BS, N = Kp - n0;
    if (N <= 0) break;
    // (2) row panel R_J,c for c >= n0: forward substitution with R_JJ^T
    for (int c = n0 + tid; c < Kp; c += blockDim.x) {
      double x[BS];
#pragma unroll
      for (int p = 0; p < BS; ++p) {
        double sacc = M[(j0 + p) * LDM + c];
#pragma unroll
        for (int q = 0; q < p; ++q) sacc = fma(-M[(j0 + q) * LDM + j0 + p], x[q], sacc);
        x[p] = sacc * rcp[j0 + p];
        M[(j0 + p) * LDM + c] = x[p];
      }
    }
    __syncthreads();
    // (3) trailing update of the upper triangle, 4 x 4 per thread
    const int n4 = N / 4;
    for (int blk = tid; blk < n4 * n4; blk += blockDim.x) {
      const int bi = blk / n4, bj = blk - bi * n4;
      if (bi > bj) continue;
      const int gi = n0 + 4 * bi, gc = n0 + 4 * bj;
      double acc[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = M[(gi + u) * LDM + gc + v];
#pragma unroll
      for (int p = 0; p < BS; ++p) {
        double ra[4], rb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          ra[u] = M[(j0 + p) * LDM + gi + u];
          rb[u] = M[(j0 + p) * LDM + gc + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] = fma(-ra[u], rb[v], acc[u][v]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (gi + u <= gc + v) M[(gi + u) * LDM + gc + v] = acc[u][v];
    }
    __syncthreads();
  }
  // R out (upper triangle; the strict lower part of M is scratch from here on)
  for (int e = tid; e < K * K; e += blockDim.x) {
    const int i = e / K, c = e - i * K;
    R[e] = c >= i ? M[i * LDM + c] : 0.0;
  }
  __syncthreads();   // R is read out before the diagonal blocks are overwritten
  // diagonal blocks -> their inverses, in place (wave w takes blocks w, w + 4, ..;
  // lanes 0..15 own columns)
  for (int Jd = wave; Jd < nbk; Jd += 4) {
    const int j0 = Jd * BS, c = lane;
    if (c < BS) {
      double x[BS];
#pragma unroll
      for (int p = BS - 1; p >= 0; --p) {
        double sacc = (p == c) ? 1.0 : 0.0;
#pragma unroll
        for (int q = p + 1; q < BS; ++q) sacc = fma(-M[(j0 + p) * LDM + j0 + q], x[q], sacc);
        x[p] = (p <= c) ? sacc * rcp[j0 + p] : 0.0;
      }
      // every lane of the wave has read the block before any lane writes it
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int p = 0; p < BS; ++p)
        if (p <= c) M[(j0 + p) * LDM + j0 + c] = x[p];
    }
  }
  __syncthreads();
  for (int I = nbk - 2; I >= 0; --I) {
    const int i0 = I * BS, n0 = i0 + BS, N = Kp - n0;
    // T[r][c] = sum_{k = n0 .. c} R[i0 + r][k] X[k][c], kept transposed at
    // M[c][i0 + r]; thread (c, r4) owns rows 4 r4 .. 4 r4 + 3 of column c
    for (int e = tid; e < 4 * N; e += blockDim.x) {
      const int r4 = e / N, c = n0 + (e - r4 * N);
      double t4[4] = {0.0, 0.0, 0.0, 0.0};
      for (int k2 = n0; k2 <= c; ++k2) {
        const double xk = M[k2 * LDM + c];
#pragma unroll
        for (int u = 0; u < 4; ++u) t4[u] = fma(M[(i0 + 4 * r4 + u) * LDM + k2], xk, t4[u]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) M[c * LDM + i0 + 4 * r4 + u] = t4[u];
    }
    __syncthreads();
    // X[i0 + r][c] = -sum_{q >= r} Xdiag[r][q] T[q][c]
    for (int e = tid; e < BS * N; e += blockDim.x) {
      const int r = e / N, c = n0 + (e - r * N);
      double sacc = 0.0;
      for (int q = r; q < BS; ++q) sacc = fma(M[(i0 + r) * LDM + i0 + q], M[c * LDM + i0 + q], sacc);
      M[(i0 + r) * LDM + c] = -sacc;
    }
    __syncthreads();
  }
  for (int e = tid; e < K * K; e += blockDim.x) {
    const int i = e / K, c = e - i * K;
    Rinv[e] = c >= i ? M[i * LDM + c] : 0.0;
  }
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

// --------------------------------------------------------------------------
// Parallel two-sided Jacobi (round-robin pairing), float64, K <= 128.
// Every workgroup runs the identical iteration on its own copy of A (in LDS)
// and accumulates the 16 rows [16*blockIdx.x, 16*blockIdx.x + 16) of the
// eigenvector matrix W.  Each round rotates K/2 disjoint pairs at once:
// A <- J^T A J, W <- W J, with the classical rotation that zeroes a_pq
// (tau = (a_qq - a_pp)/(2 a_pq), t = sign(tau)/(|tau| + sqrt(1+tau^2))).
// Stops when off(A) <= 1e-15 ||A||_F or a sweep rotates nothing.
// Output: evals[K] descending; Ws[i][rank] = W[i][col] sorted to match.
// --------------------------------------------------------------------------
constexpr int kJacRows = 16;

__device__ inline int rr_pos(int m, int r, int kpad) {
  return m == 0 ? 0 : 1 + (m - 1 + r) % (kpad - 1);
}

__device__ double block_sum(double v, double* red) {
  // 1024 threads -> 16 waves
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(1024) void k_jacobi(const double* __restrict__ H, int K,
                                                 double* __restrict__ Ws, double* __restrict__ evals,
                                                 int max_sweeps, int* status) {
  __shared__ double A[kMaxK * (kMaxK + 1)];   // row stride kpad + 1: column accesses spread banks
  __shared__ double Wl[kJacRows * kMaxK];
  __shared__ double cs[kMaxK / 2], sn[kMaxK / 2];
  __shared__ int pp[kMaxK / 2], qq[kMaxK / 2];
  __shared__ double red[16];
  __shared__ int any_rot;
  __shared__ int rank_of[kMaxK];
  const int tid = threadIdx.x;
  if (status_set(status)) return;
  const int kpad = K + (K & 1);     // index K is a dummy when K is odd
  const int npair = kpad / 2;
  const int la = kpad + 1;          // LDS row stride of A
  const int row0 = blockIdx.x * kJacRows;
  // H in batches of 8 elements per thread (all loads in flight before use)
  for (int e0 = tid; e0 < kpad * kpad; e0 += 8 * 1024) {
    double hv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + 1024 * u;
      const int i = e / kpad, j = e % kpad;
      hv[u] = (e < kpad * kpad && i < K && j < K) ? 0.5 * (H[i * K + j] + H[j * K + i]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + 1024 * u;
      if (e < kpad * kpad) A[(e / kpad) * la + (e % kpad)] = hv[u];
    }
  }
  for (int e = tid; e < kJacRows * kpad; e += blockDim.x) {
    const int r = e / kpad, j = e % kpad;
    Wl[e] = (row0 + r == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  double loc = 0.0;
  for (int e = tid; e < kpad * kpad; e += blockDim.x) {
    const int i = e / kpad, j = e % kpad;
    loc += A[i * la + j] * A[i * la + j];
  }
  const double fro = sqrt(block_sum(loc, red));
  bool converged = (K <= 1) || fro == 0.0;
  for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
    loc = 0.0;
    for (int e = tid; e < kpad * kpad; e += blockDim.x) {
      const int i = e / kpad, j = e % kpad;
      if (i != j) loc += A[i * la + j] * A[i * la + j];
    }
    const double off = sqrt(block_sum(loc, red));
    if (off <= 1e-15 * fro) {
      converged = true;
      break;
    }
    if (tid == 0) any_rot = 0;
    __syncthreads();
    for (int r = 0; r < kpad - 1; ++r) {
      if (tid < npair) {
        int p = rr_pos(tid, r, kpad), q = rr_pos(kpad - 1 - tid, r, kpad);
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < K) {
          const double apq = A[p * la + q], app = A[p * la + p], aqq = A[q * la + q];
          if (!(fabs(apq) <= 1e-300 || fabs(apq) < 0.1 * kEps * sqrt(fabs(app * aqq)))) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + hypot(1.0, tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            any_rot = 1;
          }
        }
        pp[tid] = p; qq[tid] = q; cs[tid] = c; sn[tid] = s;
      }
      __syncthreads();
      // 2x2 blocks (bi <= bj), each updated by one thread and mirrored;
      // thread t takes bi = t/16 + 64m, bj = t%16 + 16m' (no division)
      for (int bi = tid >> 4; bi < npair; bi += 64) {
        for (int bj = tid & 15; bj < npair; bj += 16) {
          if (bi > bj) continue;
          const int pi = pp[bi], qi = qq[bi], pj = pp[bj], qj = qq[bj];
          const double ci = cs[bi], si = sn[bi], cj = cs[bj], sj = sn[bj];
          if (si == 0.0 && sj == 0.0) continue;
          const double a = A[pi * la + pj], b = A[pi * la + qj];
          const double e0 = A[qi * la + pj], f = A[qi * la + qj];
          const double a1 = ci * a - si * e0, b1 = ci * b - si * f;
          const double e1 = si * a + ci * e0, f1 = si * b + ci * f;
          double a2 = cj * a1 - sj * b1, b2 = sj * a1 + cj * b1;
          double e2 = cj * e1 - sj * f1, f2 = sj * e1 + cj * f1;
          if (bi == bj) {
            A[pi * la + pi] = a2;
            A[qi * la + qi] = f2;
            A[pi * la + qi] = 0.0;
            A[qi * la + pi] = 0.0;
          } else {
            A[pi * la + pj] = a2; A[pj * la + pi] = a2;
            A[pi * la + qj] = b2; A[qj * la + pi] = b2;
            A[qi * la + pj] = e2; A[pj * la + qi] = e2;
            A[qi * la + qj] = f2; A[qj * la + qi] = f2;
          }
        }
      }
      // W rows of this workgroup: thread t takes row t/64 and pair t%64
      for (int lr = tid >> 6; lr < kJacRows; lr += 16) {
        for (int i = tid & 63; i < npair; i += 64) {
          const double s = sn[i];
          if (s == 0.0) continue;
          const double c = cs[i];
          const int p = pp[i], q = qq[i];
          const double wp = Wl[lr * kpad + p], wq = Wl[lr * kpad + q];
          Wl[lr * kpad + p] = c * wp - s * wq;
          Wl[lr * kpad + q] = s * wp + c * wq;
        }
      }
      __syncthreads();
    }
    if (!any_rot) converged = true;
    __syncthreads();
  }
  if (!converged) {
    loc = 0.0;
    for (int e = tid; e < kpad * kpad; e += blockDim.x) {
      const int i = e / kpad, j = e % kpad;
      if (i != j) loc += A[i * la + j] * A[i * la + j];
    }
    const double off = sqrt(block_sum(loc, red));
    if (off > 1e-15 * fro) {
      if (tid == 0) set_status(status, PPCA_ERR_NO_CONVERGENCE);
      return;
    }
  }
  // stable descending ranks
  for (int i = tid; i < K; i += blockDim.x) {
    const double ti = A[i * la + i];
    int rk = 0;
    for (int j = 0; j < K; ++j) {
      const double tj = A[j * la + j];
      rk += (tj > ti) || (tj == ti && j < i);
    }
    rank_of[i] = rk;
    if (blockIdx.x == 0) evals[rk] = ti;
  }
  __syncthreads();
  for (int e = tid; e < kJacRows * K; e += blockDim.x) {
    const int lr = e / K, i = e % K;
    if (row0 + lr < K) Ws[(row0 + lr) * K + rank_of[i]] = Wl[lr * kpad + i];
  }
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
  const bool flip = E[bi[0] * k + c] < 0.f;
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
                               const float* col_scale, void* vop, double* veff, hipStream_t s) {
  hipLaunchKernelGGL(k_make_operand, dim3(grid_for((int64_t)Kp * dp)), dim3(256), 0, s, V, d, K,
                     Kp, dp, (int)dtype, col_scale, vop, veff);
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
