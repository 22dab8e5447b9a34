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
// Gram partials: parts[w] = A[rows of w]^T A[rows of w], 64 rows per block.
// --------------------------------------------------------------------------
constexpr int kGramRows = 64;

template <typename T>
__global__ __launch_bounds__(256) void k_gram_part(const T* __restrict__ A, int64_t rows, int K,
                                                   int64_t lda, double* __restrict__ parts) {
  __shared__ double tile[kGramRows * kMaxK];
  const int64_t r0 = (int64_t)blockIdx.x * kGramRows;
  const int nr = (int)((rows - r0) < kGramRows ? (rows - r0) : kGramRows);
  for (int e = threadIdx.x; e < kGramRows * K; e += blockDim.x) {
    const int r = e / K, c = e % K;
    tile[r * K + c] = r < nr ? (double)A[(r0 + r) * lda + c] : 0.0;
  }
  __syncthreads();
  const int kq = (K + 3) / 4;
  double* out = parts + (int64_t)blockIdx.x * K * K;
  for (int blk = threadIdx.x; blk < kq * kq; blk += blockDim.x) {
    const int bi = blk / kq, bj = blk % kq;
    double s[4][4] = {};
    for (int r = 0; r < nr; ++r) {
      double ai[4], aj[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = 4 * bi + u, j = 4 * bj + u;
        ai[u] = i < K ? tile[r * K + i] : 0.0;
        aj[u] = j < K ? tile[r * K + j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) s[u][v] = fma(ai[u], aj[v], s[u][v]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 4 * bi + u, j = 4 * bj + v;
        if (i < K && j < K) out[i * K + j] = s[u][v];
      }
  }
}

__global__ __launch_bounds__(256) void k_sum_parts(const double* __restrict__ parts, int nparts,
                                                   int64_t count, double* __restrict__ out,
                                                   int* status) {
  bool bad = false;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += parts[(int64_t)p * count + e];
    if (!isfinite(s)) bad = true;
    out[e] = s;
  }
  if (bad) set_status(status, PPCA_ERR_NONFINITE);
}

// --------------------------------------------------------------------------
// Upper Cholesky factor R (R^T R = A) and its inverse, K <= 128, one
// workgroup of 1024 threads.  Thread (ty, tx) = (tid / 32, tid % 32) keeps the
// 4 x 4 elements (ty + 32p, tx + 32q) of the working matrix in registers.
// Right-looking factorisation, two barriers per column j:
//   (a) the owner of (j, j) checks the pivot (finite, > K * eps * |a_jj|,
//       > 0; else NOT_SPD) and publishes r_jj = sqrt(pivot);
//   (b) the owners of row j scale it, u_c = m_jc / r_jj, and publish u;
//   (c) every thread updates its trailing elements, m_ic -= u_i u_c.
// Then R goes to LDS and X = R^-1 follows from R X = I by right-looking back
// substitution (row i of X = row i of B / r_ii, then B_p -= r_pi X_i for
// p < i), one barrier per row.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_chol_inv(const double* __restrict__ A, int K,
                                                   double* __restrict__ R,
                                                   double* __restrict__ Rinv, int* status) {
  constexpr int KM = kMaxK;          // 128
  __shared__ double Rs[KM * KM];     // R (row-major) for the inverse
  __shared__ double ub[KM];          // published row of the current step
  __shared__ double xb[2][KM];       // published rows of X (double buffered)
  __shared__ double dg[KM];          // diagonal of A
  __shared__ double rd[KM];          // diagonal of R
  __shared__ int fail;
  const int tid = threadIdx.x, ty = tid >> 5, tx = tid & 31;
  if (status_set(status)) return;
  if (tid == 0) fail = 0;
  double m[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = ty + 32 * p, c = tx + 32 * q;
      m[p][q] = (i < K && c < K) ? A[i * K + c] : 0.0;
      if (i == c && i < K) dg[i] = m[p][q];
    }
  __syncthreads();
  for (int j = 0; j < K; ++j) {
    const int pj = j >> 5, oj = j & 31;
    // (a) pivot
    if (ty == oj && tx == oj) {
      double piv = 0.0;
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (p == pj && q == pj) piv = m[p][q];
      if (!(isfinite(piv) && piv > (double)K * kEps * fabs(dg[j]) && piv > 0.0)) fail = 1;
      else rd[j] = sqrt(piv);
    }
    __syncthreads();
    if (fail) {
      if (tid == 0) set_status(status, PPCA_ERR_NOT_SPD);
      return;
    }
    const double rjj = rd[j];
    // (b) row j of R
    if (ty == oj) {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        if (p != pj) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int c = tx + 32 * q;
          double v = 0.0;
          if (c == j) v = rjj;
          else if (c > j && c < K) v = m[p][q] / rjj;
          m[p][q] = v;
          if (c < K) ub[c] = v;
        }
      }
    }
    __syncthreads();
    // (c) trailing update of the elements (i, c) with i, c > j
    double ui[4], uc[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int i = ty + 32 * p;
      ui[p] = (i > j && i < K) ? ub[i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = tx + 32 * q;
      uc[q] = (c > j && c < K) ? ub[c] : 0.0;
    }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) m[p][q] = fma(-ui[p], uc[q], m[p][q]);
  }
  // R out (upper part; rows below their diagonal hold zeros from step (b))
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = ty + 32 * p, c = tx + 32 * q;
      if (i < K && c < K) {
        const double v = c >= i ? m[p][q] : 0.0;
        R[i * K + c] = v;
        Rs[i * KM + c] = v;
      }
    }
  // X = R^-1: B starts as the identity
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) m[p][q] = (ty + 32 * p == tx + 32 * q) ? 1.0 : 0.0;
  __syncthreads();
  for (int i = K - 1; i >= 0; --i) {
    const int pi = i >> 5, oi = i & 31, buf = i & 1;
    if (ty == oi) {
      const double rii = rd[i];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        if (p != pi) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int c = tx + 32 * q;
          const double v = (c >= i && c < K) ? m[p][q] / rii : 0.0;
          m[p][q] = v;
          if (c < K) xb[buf][c] = v;
        }
      }
    }
    __syncthreads();
    double xc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = tx + 32 * q;
      xc[q] = (c >= i && c < K) ? xb[buf][c] : 0.0;
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int r = ty + 32 * p;
      if (r < i) {
        const double rpi = Rs[r * KM + i];
#pragma unroll
        for (int q = 0; q < 4; ++q) m[p][q] = fma(-rpi, xc[q], m[p][q]);
      }
    }
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = ty + 32 * p, c = tx + 32 * q;
      if (i < K && c < K) Rinv[i * K + c] = c >= i ? m[p][q] : 0.0;
    }
}

// --------------------------------------------------------------------------
// out = A * Rinv for upper-triangular Rinv (K x K), 16 rows per block.
// --------------------------------------------------------------------------
constexpr int kTrmmRows = 16;

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_trmm(const TI* __restrict__ A, int64_t rows, int K,
                                              int64_t lda, const double* __restrict__ Rinv,
                                              TO* __restrict__ out, int64_t ldo, int* status) {
  __shared__ double Rs[kMaxK * kMaxK];
  __shared__ double As[kTrmmRows * kMaxK];
  if (status_set(status)) return;
  const int64_t r0 = (int64_t)blockIdx.x * kTrmmRows;
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) Rs[e] = Rinv[e];
  for (int e = threadIdx.x; e < kTrmmRows * K; e += blockDim.x) {
    const int r = e / K, c = e % K;
    As[e] = (r0 + r < rows) ? (double)A[(r0 + r) * lda + c] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kTrmmRows * K; e += blockDim.x) {
    const int r = e / K, c = e % K;
    if (r0 + r >= rows) continue;
    double s = 0.0;
    for (int p = 0; p <= c; ++p) s = fma(As[r * K + p], Rs[p * K + c], s);
    out[(r0 + r) * ldo + c] = (TO)s;
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
  __shared__ double A[kMaxK * kMaxK];
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
  const int row0 = blockIdx.x * kJacRows;
  for (int e = tid; e < kpad * kpad; e += blockDim.x) {
    const int i = e / kpad, j = e % kpad;
    A[e] = (i < K && j < K) ? 0.5 * (H[i * K + j] + H[j * K + i]) : 0.0;
  }
  for (int e = tid; e < kJacRows * kpad; e += blockDim.x) {
    const int r = e / kpad, j = e % kpad;
    Wl[e] = (row0 + r == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  double loc = 0.0;
  for (int e = tid; e < kpad * kpad; e += blockDim.x) loc += A[e] * A[e];
  const double fro = sqrt(block_sum(loc, red));
  bool converged = (K <= 1) || fro == 0.0;
  for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
    loc = 0.0;
    for (int e = tid; e < kpad * kpad; e += blockDim.x) {
      const int i = e / kpad, j = e % kpad;
      if (i != j) loc += A[e] * A[e];
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
          const double apq = A[p * kpad + q], app = A[p * kpad + p], aqq = A[q * kpad + q];
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
      // 2x2 blocks (bi <= bj), each updated by one thread and mirrored
      for (int e = tid; e < npair * npair; e += blockDim.x) {
        const int bi = e / npair, bj = e % npair;
        if (bi > bj) continue;
        const int pi = pp[bi], qi = qq[bi], pj = pp[bj], qj = qq[bj];
        const double ci = cs[bi], si = sn[bi], cj = cs[bj], sj = sn[bj];
        if (si == 0.0 && sj == 0.0) continue;
        const double a = A[pi * kpad + pj], b = A[pi * kpad + qj];
        const double e0 = A[qi * kpad + pj], f = A[qi * kpad + qj];
        const double a1 = ci * a - si * e0, b1 = ci * b - si * f;
        const double e1 = si * a + ci * e0, f1 = si * b + ci * f;
        double a2 = cj * a1 - sj * b1, b2 = sj * a1 + cj * b1;
        double e2 = cj * e1 - sj * f1, f2 = sj * e1 + cj * f1;
        if (bi == bj) {
          b2 = 0.0;
          e2 = 0.0;
          A[pi * kpad + pi] = a2;
          A[qi * kpad + qi] = f2;
          A[pi * kpad + qi] = 0.0;
          A[qi * kpad + pi] = 0.0;
        } else {
          A[pi * kpad + pj] = a2; A[pj * kpad + pi] = a2;
          A[pi * kpad + qj] = b2; A[qj * kpad + pi] = b2;
          A[qi * kpad + pj] = e2; A[pj * kpad + qi] = e2;
          A[qi * kpad + qj] = f2; A[qj * kpad + qi] = f2;
        }
      }
      for (int e = tid; e < kJacRows * npair; e += blockDim.x) {
        const int lr = e / npair, i = e % npair;
        const double s = sn[i];
        if (s == 0.0) continue;
        const double c = cs[i];
        const int p = pp[i], q = qq[i];
        const double wp = Wl[lr * kpad + p], wq = Wl[lr * kpad + q];
        Wl[lr * kpad + p] = c * wp - s * wq;
        Wl[lr * kpad + q] = s * wp + c * wq;
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
      if (i != j) loc += A[e] * A[e];
    }
    const double off = sqrt(block_sum(loc, red));
    if (off > 1e-15 * fro) {
      if (tid == 0) set_status(status, PPCA_ERR_NO_CONVERGENCE);
      return;
    }
  }
  // stable descending ranks
  for (int i = tid; i < K; i += blockDim.x) {
    const double ti = A[i * kpad + i];
    int rk = 0;
    for (int j = 0; j < K; ++j) {
      const double tj = A[j * kpad + j];
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

int gram_parts(int64_t rows) { return (int)cdiv(rows, kGramRows); }

hipError_t launch_gram(const void* A, bool in_f64, int64_t rows, int K, int64_t lda, double* parts,
                       double* out, int* status, hipStream_t s) {
  const int np = gram_parts(rows);
  if (in_f64)
    hipLaunchKernelGGL(k_gram_part<double>, dim3(np), dim3(256), 0, s, (const double*)A, rows, K,
                       lda, parts);
  else
    hipLaunchKernelGGL(k_gram_part<float>, dim3(np), dim3(256), 0, s, (const float*)A, rows, K,
                       lda, parts);
  hipLaunchKernelGGL(k_sum_parts, dim3(grid_for((int64_t)K * K)), dim3(256), 0, s, parts, np,
                     (int64_t)K * K, out, status);
  return hipGetLastError();
}

hipError_t launch_chol_inv(const double* A, int K, double* R, double* Rinv, int* status,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(1024), 0, s, A, K, R, Rinv, status);
  return hipGetLastError();
}

hipError_t launch_trmm(const void* A, bool in_f64, int64_t rows, int K, int64_t lda,
                       const double* Rinv, void* out, bool out_f64, int64_t ldo, int* status,
                       hipStream_t s) {
  const dim3 grid((unsigned)cdiv(rows, kTrmmRows));
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
