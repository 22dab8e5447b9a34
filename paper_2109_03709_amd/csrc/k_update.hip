// Minibatch updates of the SGD-style primings, applied to the d x K float32
// directions V after one streaming pass has produced Z = X_b^T X_b V' and
// G = V'^T X_b^T X_b V' (both unnormalised sums over the b rows).
//
//  Sanger / generalised Oja (Sec. 2.2):  g = (Z - V triu(G)) / b
//  EigenGame (Sec. 2.3, eqs. (1)-(3)):   grad = (2/b) Z R, R = I, R_ij = -G_ij / G_ii (i < j),
//                                        Riemannian projection, step, unit-norm columns.
//  Optional momentum (training setup of Sec. 5): buf <- mu buf + g,
//  step = g + mu buf (Nesterov) or buf.
#include "ppca_common.h"

namespace ppca {

namespace {

// Thread layout shared by the update kernels: with ng = 256 / K row groups,
// thread t < ng * K owns column c = t % K and row group g = t / K; a block covers
// rb = ng * kRowsPerThread rows and the thread handles rows g + ng * q of it.
// The 256 - ng * K spare threads (K not a power of two) load like group ng - 1
// but store nothing.  All loads are unconditional (row indices clamped to d - 1)
// so that they issue back to back.  Reductions over rows run in a fixed order
// (rows of a thread, then groups, then blocks): results do not depend on timing.
constexpr int kThreads = 256;
constexpr int kRowsPerThread = 8;

__host__ __device__ inline int row_groups(int K) { return kThreads / K; }
__host__ __device__ inline int block_rows(int K) { return row_groups(K) * kRowsPerThread; }

struct Lane {
  int c, g, ng, rb;
  bool act;
  int64_t j0;
  __device__ Lane(int K) {
    const int t = threadIdx.x;
    ng = row_groups(K);
    rb = ng * kRowsPerThread;
    c = t % K;
    g = min(t / K, ng - 1);
    act = t < ng * K;
    j0 = (int64_t)blockIdx.x * rb;
  }
  __device__ int64_t row(int q) const { return j0 + g + ng * q; }
  __device__ int lrow(int q) const { return g + ng * q; }
};

__device__ inline int64_t clamp_row(int64_t j, int64_t d) { return j < d ? j : d - 1; }

__device__ inline bool status_set(const int* status) {
  return *reinterpret_cast<const volatile int*>(status) != 0;
}

__device__ inline double momentum_step(double g, double mu, int nesterov, float* mom,
                                       int64_t idx) {
  if (mu == 0.0) return g;
  const double buf = mu * (double)mom[idx] + g;
  mom[idx] = (float)buf;
  return nesterov ? g + mu * buf : buf;
}

// out[c] = sum over w < nblk of part[w * K + c], for c < K (LDS result; scr
// holds kThreads doubles).  Loads go out eight at a time.
__device__ inline void sum_partials(const double* __restrict__ part, int nblk, int K,
                                    const Lane& L, double* scr, double* out) {
  const int t = threadIdx.x;
  double s = 0.0;
  int w = L.g;
  for (; w + 7 * L.ng < nblk; w += 8 * L.ng) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(w + u * L.ng) * K + L.c];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; w < nblk; w += L.ng) s += part[(int64_t)w * K + L.c];
  if (L.act) scr[t] = s;
  __syncthreads();
  if (t < K) {
    double r = 0.0;
    for (int g = 0; g < L.ng; ++g) r += scr[g * K + t];
    out[t] = r;
  }
  __syncthreads();
}

// Many blocks (large d): the column sums of the per-block partials are formed
// once, by K workgroups (workgroup c: thread t adds blocks t, t + 256, ... in
// order, then a fixed tree), instead of by every block of the next kernel.
constexpr int kDirectPartials = 64;   // up to this many blocks each block sums them itself

__global__ __launch_bounds__(kThreads) void k_sum_cols(const double* __restrict__ part, int nblk,
                                                       int K, double* __restrict__ out) {
  __shared__ double sh[kThreads];
  const int c = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  for (int w = t; w < nblk; w += kThreads) s += part[(int64_t)w * K + c];
  sh[t] = s;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if (t < h) sh[t] += sh[t + h];
    __syncthreads();
  }
  if (t == 0) out[c] = sh[0];
}

// the column sums of part: from the precomputed sums when there are many
// blocks, else summed here (LDS result)
__device__ inline void column_sums(const double* __restrict__ part,
                                   const double* __restrict__ pre, int nblk, int K,
                                   const Lane& L, double* scr, double* out) {
  if (pre) {
    if ((int)threadIdx.x < K) out[threadIdx.x] = pre[threadIdx.x];
    __syncthreads();
  } else {
    sum_partials(part, nblk, K, L, scr, out);
  }
}

// Per-block column sums of the thread values (fixed order) -> part[blk * K + c].
__device__ inline void block_column_sum(double val, int K, const Lane& L, double* scr,
                                        double* __restrict__ part) {
  const int t = threadIdx.x;
  if (L.act) scr[t] = val;
  __syncthreads();
  if (t < K) {
    double s = 0.0;
    for (int g = 0; g < L.ng; ++g) s += scr[g * K + t];
    part[(int64_t)blockIdx.x * K + t] = s;
  }
}

// Sanger / generalised Oja step.  LDS: Gs [K][K] f64 (upper triangle of G, zeros
// below) | Vs [rb][K] f32 (the block's rows of V).
__global__ __launch_bounds__(kThreads) void k_sanger(float* __restrict__ V,
                                                     const float* __restrict__ Z,
                                                     const double* __restrict__ G, int64_t d,
                                                     int K, int b, double eta, double mu,
                                                     int nesterov, float* __restrict__ mom,
                                                     int* status) {
  extern __shared__ double lds[];
  double* Gs = lds;
  const Lane L(K);
  float* Vs = reinterpret_cast<float*>(lds + K * K);
  const int c = L.c;
  double z[kRowsPerThread];
  float v[kRowsPerThread];
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q) {
    const int64_t jc = clamp_row(L.row(q), d);
    z[q] = (double)Z[jc * K + c];
    v[q] = V[jc * K + c];
  }
  // rows i = g, g + ng, ... of G, eight loads in flight (clamped index)
  for (int i0 = L.g; i0 < K; i0 += 8 * L.ng) {
    double gv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) gv[u] = G[min(i0 + u * L.ng, K - 1) * K + c];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * L.ng;
      if (L.act && i < K) Gs[i * K + c] = i <= c ? gv[u] : 0.0;
    }
  }
  if (L.act) {
#pragma unroll
    for (int q = 0; q < kRowsPerThread; ++q) Vs[L.lrow(q) * K + c] = v[q];
  }
  const bool stop = status_set(status);
  __syncthreads();
  if (stop || !L.act) return;
  // s = Z_jc - sum_{i <= c} V_ji G_ic, terms in order of i (zeros past c add nothing)
  for (int i = 0; i < K; ++i) {
    const double gi = Gs[i * K + c];
#pragma unroll
    for (int q = 0; q < kRowsPerThread; ++q)
      z[q] = fma(-(double)Vs[L.lrow(q) * K + i], gi, z[q]);
  }
  const double inv_b = 1.0 / (double)b;
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q) {
    const int64_t j = L.row(q);
    if (j >= d) continue;
    const double step = momentum_step(z[q] * inv_b, mu, nesterov, mom, j * K + c);
    V[j * K + c] = (float)((double)v[q] + eta * step);
  }
}

// EigenGame update in three passes over the rows of V and Z, none of which
// stores the gradient or the unnormalised step (both are recomputed, with the
// same arithmetic, from V, Z and G in every pass):
//   k_eg_dots   per-block partial dots v_c . grad_c;
//   k_eg_norms  vn = v + eta step(grad - (v . grad) v), per-block partial
//               squared norms (the momentum buffer is read, not written);
//   k_eg_apply  the same vn, V <- vn / |vn|, the momentum buffer, and (when
//               vop is given) the next step's MFMA operand of the new V.
// grad = (2/b) Z R with R_ii = 1, R_ic = -G_ic / G_ii (i < c), else 0.
// LDS (dynamic): Rs [K][K] f64 | scr [kThreads] f64 | Zs [rb][K] f32.

// Loads this thread's rows of V and the block's rows of Z, builds R, and
// returns the gradient rows in gr (valid where L.act and the row is < d).
// Returns false (in every thread) when the status word is set.
__device__ inline bool eg_grad_rows(const float* __restrict__ V, const float* __restrict__ Z,
                                    const double* __restrict__ G, int64_t d, int K, int b,
                                    const Lane& L, double* Rs, float* Zs, const int* status,
                                    float (&v)[kRowsPerThread], double (&gr)[kRowsPerThread]) {
  const int c = L.c;
  float z[kRowsPerThread];
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q) {
    const int64_t jc = clamp_row(L.row(q), d);
    z[q] = Z[jc * K + c];
    v[q] = V[jc * K + c];
  }
  // R_ic for rows i = g, g + ng, ..., eight row pairs of loads in flight
  for (int i0 = L.g; i0 < K; i0 += 8 * L.ng) {
    double gii[8], gic[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = min(i0 + u * L.ng, K - 1);
      gii[u] = G[i * K + i];
      gic[u] = G[i * K + c];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * L.ng;
      const double qv = -gic[u] / gii[u];
      const double r = (i < c && gii[u] > 1e-300) ? qv : (i == c ? 1.0 : 0.0);
      if (L.act && i < K) Rs[i * K + c] = r;
    }
  }
  if (L.act) {
#pragma unroll
    for (int q = 0; q < kRowsPerThread; ++q) Zs[L.lrow(q) * K + c] = L.row(q) < d ? z[q] : 0.f;
  }
  const bool stop = status_set(status);
  __syncthreads();
  if (stop) return false;
  double s[kRowsPerThread];
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q) s[q] = 0.0;
  for (int i = 0; i < K; ++i) {
    const double ri = Rs[i * K + c];
#pragma unroll
    for (int q = 0; q < kRowsPerThread; ++q) s[q] = fma((double)Zs[L.lrow(q) * K + i], ri, s[q]);
  }
  const double sc = 2.0 / (double)b;
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q) gr[q] = sc * s[q];
  return true;
}

// The step of momentum_step without writing the buffer.
__device__ inline double momentum_peek(double g, double mu, int nesterov, const float* mom,
                                       int64_t idx) {
  if (mu == 0.0) return g;
  const double buf = mu * (double)mom[idx] + g;
  return nesterov ? g + mu * buf : buf;
}

__global__ __launch_bounds__(kThreads) void k_eg_dots(const float* __restrict__ V,
                                                      const float* __restrict__ Z,
                                                      const double* __restrict__ G, int64_t d,
                                                      int K, int b, double* __restrict__ pdot,
                                                      int* status) {
  extern __shared__ double lds[];
  const Lane L(K);
  double* Rs = lds;
  double* scr = lds + K * K;
  float* Zs = reinterpret_cast<float*>(scr + kThreads);
  float v[kRowsPerThread];
  double gr[kRowsPerThread];
  if (!eg_grad_rows(V, Z, G, d, K, b, L, Rs, Zs, status, v, gr)) return;
  double dot = 0.0;
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q)
    if (L.act && L.row(q) < d) dot += (double)v[q] * gr[q];
  block_column_sum(dot, K, L, scr, pdot);
}

__global__ __launch_bounds__(kThreads) void k_eg_norms(const float* __restrict__ V,
                                                       const float* __restrict__ Z,
                                                       const double* __restrict__ G, int64_t d,
                                                       int K, int b, const double* __restrict__ pdot,
                                                       const double* __restrict__ pdot_sum,
                                                       int nblk, double eta, double mu,
                                                       int nesterov, const float* __restrict__ mom,
                                                       double* __restrict__ pnorm, int* status) {
  extern __shared__ double lds[];
  __shared__ double dots[kMaxK];
  const Lane L(K);
  double* Rs = lds;
  double* scr = lds + K * K;
  float* Zs = reinterpret_cast<float*>(scr + kThreads);
  float v[kRowsPerThread];
  double gr[kRowsPerThread];
  if (!eg_grad_rows(V, Z, G, d, K, b, L, Rs, Zs, status, v, gr)) return;
  column_sums(pdot, pdot_sum, nblk, K, L, scr, dots);
  const int c = L.c;
  double sq = 0.0;
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q) {
    const int64_t j = L.row(q);
    if (L.act && j < d) {
      const double vq = (double)v[q];
      const double gq = gr[q] - dots[c] * vq;
      const double vn = vq + eta * momentum_peek(gq, mu, nesterov, mom, j * K + c);
      sq += vn * vn;
    }
  }
  block_column_sum(sq, K, L, scr, pnorm);
}

__global__ __launch_bounds__(kThreads) void k_eg_apply(float* __restrict__ V,
                                                       const float* __restrict__ Z,
                                                       const double* __restrict__ G, int64_t d,
                                                       int K, int b, const double* __restrict__ pdot,
                                                       const double* __restrict__ pnorm,
                                                       const double* __restrict__ sums, int nblk,
                                                       double eta, double mu, int nesterov,
                                                       float* __restrict__ mom, void* __restrict__ vop,
                                                       int64_t dp, int dtype,
                                                       const float* __restrict__ scale,
                                                       int* status) {
  extern __shared__ double lds[];
  __shared__ double dots[kMaxK], nrm[kMaxK];
  const Lane L(K);
  double* Rs = lds;
  double* scr = lds + K * K;
  float* Zs = reinterpret_cast<float*>(scr + kThreads);
  float v[kRowsPerThread];
  double gr[kRowsPerThread];
  if (!eg_grad_rows(V, Z, G, d, K, b, L, Rs, Zs, status, v, gr)) return;
  column_sums(pdot, sums, nblk, K, L, scr, dots);
  column_sums(pnorm, sums ? sums + K : nullptr, nblk, K, L, scr, nrm);
  if (threadIdx.x < K) {
    const double s = nrm[threadIdx.x];
    if (!(s > 0.0) || !isfinite(s)) set_status(status, PPCA_ERR_NONFINITE);
  }
  if (!L.act) return;
  const int c = L.c;
  const double ic = 1.0 / sqrt(nrm[c]);
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q) {
    const int64_t j = L.row(q);
    if (j < d) {
      const double vq = (double)v[q];
      const double gq = gr[q] - dots[c] * vq;
      const double vn = vq + eta * momentum_step(gq, mu, nesterov, mom, j * K + c);
      const float vf = (float)(vn * ic);
      V[j * K + c] = vf;
      if (vop) {
        // the operand entry k_make_operand would write for this V
        const int64_t e = (int64_t)c * dp + j;
        if (dtype == PPCA_F32) {
          reinterpret_cast<float*>(vop)[e] = vf;
        } else {
          const float sv = dtype == PPCA_FP8_E4M3 ? scale[j] * vf : vf;
          reinterpret_cast<uint16_t*>(vop)[e] = (uint16_t)f32_to_bf16_bits(sv);
        }
      }
    }
  }
}

__global__ void k_copy_f32(const float* __restrict__ s, float* __restrict__ d, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    d[e] = s[e];
}

}  // namespace

int eigengame_blocks(int64_t d, int K) { return (int)cdiv(d, block_rows(K)); }

hipError_t launch_sanger_update(float* V, const float* Z, const double* G, int64_t d, int K, int b,
                                double eta, double mu, int nesterov, float* mom, int* status,
                                hipStream_t s) {
  const size_t lds = (size_t)K * K * sizeof(double) + (size_t)block_rows(K) * K * sizeof(float);
  hipLaunchKernelGGL(k_sanger, dim3((unsigned)cdiv(d, block_rows(K))), dim3(kThreads), lds, s, V,
                     Z, G, d, K, b, eta, mu, nesterov, mom, status);
  return hipGetLastError();
}

size_t eigengame_scratch_doubles(int64_t d, int K) {
  return (size_t)(2 * (int64_t)eigengame_blocks(d, K) * K + 2 * K);
}

// scratch layout: pdot [nblk*K] | pnorm [nblk*K] | pdot sums [K] | pnorm sums [K]
// (float64).  vop (optional): the operand of the new V, [Kp][dp] (its padding
// is left as it is: zero from the operand built before the first step).
hipError_t launch_eigengame_update(float* V, const float* Z, const double* G, int64_t d, int K,
                                   int b, double eta, double mu, int nesterov, float* mom,
                                   double* scratch, void* vop, int64_t dp, int32_t dtype,
                                   const float* col_scale, int* status, hipStream_t s) {
  const int nblk = eigengame_blocks(d, K);
  double* pdot = scratch;
  double* pnorm = pdot + (int64_t)nblk * K;
  double* sums = pnorm + (int64_t)nblk * K;
  const bool two_level = nblk > kDirectPartials;
  const size_t lds = ((size_t)K * K + kThreads) * sizeof(double) +
                     (size_t)block_rows(K) * K * sizeof(float);
  hipLaunchKernelGGL(k_eg_dots, dim3(nblk), dim3(kThreads), lds, s, V, Z, G, d, K, b, pdot,
                     status);
  if (two_level) hipLaunchKernelGGL(k_sum_cols, dim3(K), dim3(kThreads), 0, s, pdot, nblk, K, sums);
  hipLaunchKernelGGL(k_eg_norms, dim3(nblk), dim3(kThreads), lds, s, V, Z, G, d, K, b, pdot,
                     two_level ? (const double*)sums : nullptr, nblk, eta, mu, nesterov,
                     (const float*)mom, pnorm, status);
  if (two_level)
    hipLaunchKernelGGL(k_sum_cols, dim3(K), dim3(kThreads), 0, s, pnorm, nblk, K, sums + K);
  hipLaunchKernelGGL(k_eg_apply, dim3(nblk), dim3(kThreads), lds, s, V, Z, G, d, K, b, pdot, pnorm,
                     two_level ? (const double*)sums : nullptr, nblk, eta, mu, nesterov, mom, vop,
                     dp, (int)dtype, col_scale, status);
  return hipGetLastError();
}

hipError_t launch_copy_f32(const float* src, float* dst, int64_t count, hipStream_t s) {
  int64_t g = cdiv(count, 256);
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_copy_f32, dim3(g), dim3(256), 0, s, src, dst, count);
  return hipGetLastError();
}

}  // namespace ppca
