// Minibatch updates of the SGD-style primings, applied to the d x K float32
// directions V after one streaming pass has produced Z = X_b^T X_b V' and
// G = V'^T X_b^T X_b V' (both unnormalised sums over the b rows).
//
//  Sanger / generalised Oja (Sec. 2.2):  g = (Z - V triu(G)) / b
//  EigenGame (Sec. 2.3, eqs. (1)-(3)):   grad = (2/b) Z R, R = I, R_ij = -G_ij / G_ii (i < j),
//                                        Riemannian projection, step, unit-norm columns.
//  Optional momentum (training setup of Sec. 5): buf <- mu buf + g,
//  step = g + mu buf (Nesterov) or buf.
//
// Both updates also write the MFMA operand of the new V (when asked), so the
// next minibatch pass needs no operand kernel of its own.
#include "ppca_common.h"

namespace ppca {

namespace {

// Thread layout shared by the update kernels: with ng = 256 / K row groups,
// thread t < ng * K owns column c = t % K and row group g = t / K; a block covers
// rb = ng * RPT rows and the thread handles rows g + ng * q of it (q < RPT).
// RPT (rows per thread) is 8 for large d and drops to 4, 2 or 1 when d is
// small, so that the update still runs on about 256 workgroups.
// The 256 - ng * K spare threads (K not a power of two) load like group ng - 1
// but store nothing.  All loads are unconditional (row indices clamped to d - 1)
// so that they issue back to back.  Reductions over rows run in a fixed order
// (rows of a thread, then groups, then blocks): results do not depend on timing.
constexpr int kThreads = 256;
constexpr int kMaxRPT = 8;

__host__ __device__ inline int row_groups(int K) { return kThreads / K; }

template <int RPT>
struct Lane {
  int c, g, ng, rb;
  bool act;
  int64_t j0;
  __device__ Lane(int K) {
    const int t = threadIdx.x;
    ng = row_groups(K);
    rb = ng * RPT;
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

// The operand entry (c, j) of the new value vf of V: what k_make_operand
// writes for it (float32 data: vf; else bf16 of vf, of s_j vf for fp8).
__device__ inline void write_operand(void* vop, int64_t dp, int dtype, const float* scale, int c,
                                     int64_t j, float vf) {
  const int64_t e = (int64_t)c * dp + j;
  if (dtype == PPCA_F32) {
    reinterpret_cast<float*>(vop)[e] = vf;
  } else {
    const float sv = dtype == PPCA_FP8_E4M3 ? scale[j] * vf : vf;
    reinterpret_cast<uint16_t*>(vop)[e] = (uint16_t)f32_to_bf16_bits(sv);
  }
}

// out[c] = sum over w < nblk of part[w * ld + c], for c < K (LDS result; scr
// holds kThreads doubles).  Loads go out eight at a time.
template <int RPT>
__device__ inline void sum_partials(const double* __restrict__ part, int nblk, int K, int64_t ld,
                                    const Lane<RPT>& L, double* scr, double* out) {
  const int t = threadIdx.x;
  double s = 0.0;
  int w = L.g;
  for (; w + 7 * L.ng < nblk; w += 8 * L.ng) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(w + u * L.ng) * ld + L.c];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; w < nblk; w += L.ng) s += part[(int64_t)w * ld + L.c];
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
// once, by one workgroup per column (thread t adds blocks t, t + 256, ... in
// order, eight loads in flight, then a fixed tree), instead of by every block
// of the next kernel.
constexpr int kDirectPartials = 64;   // up to this many blocks each block sums them itself

__global__ __launch_bounds__(kThreads) void k_sum_cols(const double* __restrict__ part, int nblk,
                                                       int ncol, double* __restrict__ out) {
  __shared__ double sh[kThreads];
  const int c = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  int w = t;
  for (; w + 7 * kThreads < nblk; w += 8 * kThreads) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(w + u * kThreads) * ncol + c];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; w < nblk; w += kThreads) s += part[(int64_t)w * ncol + c];
  sh[t] = s;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if (t < h) sh[t] += sh[t + h];
    __syncthreads();
  }
  if (t == 0) out[c] = sh[0];
}

// Per-block column sums of the thread values (fixed order) -> part[c]
// (part already offset to this block's row of partials).  Starts with a
// barrier, so that calls may follow one another on the same scr.
template <int RPT>
__device__ inline void block_column_sum(double val, int K, const Lane<RPT>& L, double* scr,
                                        double* __restrict__ part) {
  const int t = threadIdx.x;
  __syncthreads();
  if (L.act) scr[t] = val;
  __syncthreads();
  if (t < K) {
    double s = 0.0;
    for (int g = 0; g < L.ng; ++g) s += scr[g * K + t];
    part[t] = s;
  }
}

// Sanger / generalised Oja step.  LDS: Gs [K][K] f64 (upper triangle of G, zeros
// below) | Vs [rb][K] f32 (the block's rows of V).
template <int RPT>
__global__ __launch_bounds__(kThreads) void k_sanger(float* __restrict__ V,
                                                     const float* __restrict__ Z,
                                                     const double* __restrict__ G, int64_t d,
                                                     int K, int b, double eta, double mu,
                                                     int nesterov, float* __restrict__ mom,
                                                     void* __restrict__ vop, int64_t dp, int dtype,
                                                     const float* __restrict__ scale,
                                                     int* status) {
  extern __shared__ double lds[];
  double* Gs = lds;
  const Lane<RPT> L(K);
  float* Vs = reinterpret_cast<float*>(lds + K * K);
  const int c = L.c;
  double z[RPT];
  float v[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
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
    for (int q = 0; q < RPT; ++q) Vs[L.lrow(q) * K + c] = v[q];
  }
  const bool stop = status_set(status);
  __syncthreads();
  if (stop || !L.act) return;
  // s = Z_jc - sum_{i <= c} V_ji G_ic, terms in order of i (zeros past c add nothing)
  for (int i = 0; i < K; ++i) {
    const double gi = Gs[i * K + c];
#pragma unroll
    for (int q = 0; q < RPT; ++q) z[q] = fma(-(double)Vs[L.lrow(q) * K + i], gi, z[q]);
  }
  const double inv_b = 1.0 / (double)b;
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t j = L.row(q);
    if (j >= d) continue;
    const double step = momentum_step(z[q] * inv_b, mu, nesterov, mom, j * K + c);
    const float vf = (float)((double)v[q] + eta * step);
    V[j * K + c] = vf;
    if (vop) write_operand(vop, dp, dtype, scale, c, j, vf);
  }
}

// EigenGame update in two passes over the rows of V and Z; neither stores the
// gradient (it is recomputed, with the same arithmetic, from V, Z and G):
//   k_eg_sums   per block and column: S_vv = sum v^2, S_gg = sum g^2,
//               S_mm = sum m^2, S_vg = sum v g, S_vm = sum v m, S_gm = sum g m
//               (g the gradient, m the momentum buffer, zero without momentum);
//   k_eg_apply  dot = S_vg; the step is vn = a v + p g + r m with
//               a = 1 - eta alpha dot, p = eta alpha, r = eta beta, where
//               alpha, beta = 1, mu (heavy ball), 1 + mu, mu^2 (Nesterov),
//               beta = 0 without momentum; so
//               |vn|^2 = a^2 S_vv + p^2 S_gg + r^2 S_mm + 2ap S_vg + 2ar S_vm
//                        + 2pr S_gm,
//               then V <- vn / |vn|, the momentum buffer, and (when vop is
//               given) the next step's operand.
// grad = (2/b) Z R with R_ii = 1, R_ic = -G_ic / G_ii (i < c), else 0.
// LDS (dynamic): Rs [K][K] f64 | scr [kThreads] f64 | Zs [rb][K] f32.
constexpr int kEgSums = 6;

// Loads this thread's rows of V and the block's rows of Z, builds R, and
// returns the gradient rows in gr (valid where L.act and the row is < d).
// Returns false (in every thread) when the status word is set.
template <int RPT>
__device__ inline bool eg_grad_rows(const float* __restrict__ V, const float* __restrict__ Z,
                                    const double* __restrict__ G, int64_t d, int K, int b,
                                    const Lane<RPT>& L, double* Rs, float* Zs, const int* status,
                                    float (&v)[RPT], double (&gr)[RPT]) {
  const int c = L.c;
  float z[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
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
    for (int q = 0; q < RPT; ++q) Zs[L.lrow(q) * K + c] = L.row(q) < d ? z[q] : 0.f;
  }
  const bool stop = status_set(status);
  __syncthreads();
  if (stop) return false;
  double s[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) s[q] = 0.0;
  for (int i = 0; i < K; ++i) {
    const double ri = Rs[i * K + c];
#pragma unroll
    for (int q = 0; q < RPT; ++q) s[q] = fma((double)Zs[L.lrow(q) * K + i], ri, s[q]);
  }
  const double sc = 2.0 / (double)b;
#pragma unroll
  for (int q = 0; q < RPT; ++q) gr[q] = sc * s[q];
  return true;
}

// part: [nblk][kEgSums][K]; mom null without momentum
template <int RPT>
__global__ __launch_bounds__(kThreads) void k_eg_sums(const float* __restrict__ V,
                                                      const float* __restrict__ Z,
                                                      const double* __restrict__ G, int64_t d,
                                                      int K, int b, const float* __restrict__ mom,
                                                      double* __restrict__ part, int* status) {
  extern __shared__ double lds[];
  const Lane<RPT> L(K);
  double* Rs = lds;
  double* scr = lds + K * K;
  float* Zs = reinterpret_cast<float*>(scr + kThreads);
  float v[RPT];
  double gr[RPT];
  if (!eg_grad_rows(V, Z, G, d, K, b, L, Rs, Zs, status, v, gr)) return;
  double s[kEgSums] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t j = L.row(q);
    if (L.act && j < d) {
      const double vq = (double)v[q], gq = gr[q];
      const double mq = mom ? (double)mom[j * K + L.c] : 0.0;
      s[0] = fma(vq, vq, s[0]);
      s[1] = fma(gq, gq, s[1]);
      s[2] = fma(mq, mq, s[2]);
      s[3] = fma(vq, gq, s[3]);
      s[4] = fma(vq, mq, s[4]);
      s[5] = fma(gq, mq, s[5]);
    }
  }
  double* pb = part + (int64_t)blockIdx.x * kEgSums * K;
#pragma unroll
  for (int u = 0; u < kEgSums; ++u) block_column_sum(s[u], K, L, scr, pb + u * K);
}

template <int RPT>
__global__ __launch_bounds__(kThreads) void k_eg_apply(float* __restrict__ V,
                                                       const float* __restrict__ Z,
                                                       const double* __restrict__ G, int64_t d,
                                                       int K, int b, const double* __restrict__ part,
                                                       const double* __restrict__ sums, int nblk,
                                                       double eta, double mu, int nesterov,
                                                       float* __restrict__ mom, void* __restrict__ vop,
                                                       int64_t dp, int dtype,
                                                       const float* __restrict__ scale,
                                                       int* status) {
  extern __shared__ double lds[];
  __shared__ double S[kEgSums][kMaxK];
  __shared__ double coef[2][kMaxK];   // dot and 1 / |vn| per column
  const Lane<RPT> L(K);
  double* Rs = lds;
  double* scr = lds + K * K;
  float* Zs = reinterpret_cast<float*>(scr + kThreads);
  float v[RPT];
  double gr[RPT];
  if (!eg_grad_rows(V, Z, G, d, K, b, L, Rs, Zs, status, v, gr)) return;
  if (sums) {
    for (int e = threadIdx.x; e < kEgSums * K; e += kThreads) S[e / K][e % K] = sums[e];
    __syncthreads();
  } else {
#pragma unroll
    for (int u = 0; u < kEgSums; ++u)
      sum_partials(part + u * K, nblk, K, (int64_t)kEgSums * K, L, scr, S[u]);
  }
  const double alpha = nesterov ? 1.0 + mu : 1.0;
  const double beta = mu != 0.0 ? (nesterov ? mu * mu : mu) : 0.0;
  if ((int)threadIdx.x < K) {
    const int cc = threadIdx.x;
    const double dot = S[3][cc];
    const double a = 1.0 - eta * alpha * dot, p = eta * alpha, r = eta * beta;
    const double n2 = a * a * S[0][cc] + p * p * S[1][cc] + r * r * S[2][cc] +
                      2.0 * a * p * S[3][cc] + 2.0 * a * r * S[4][cc] + 2.0 * p * r * S[5][cc];
    if (!(n2 > 0.0) || !isfinite(n2)) set_status(status, PPCA_ERR_NONFINITE);
    coef[0][cc] = dot;
    coef[1][cc] = 1.0 / sqrt(n2);
  }
  __syncthreads();
  if (!L.act) return;
  const int c = L.c;
  const double dot = coef[0][c], ic = coef[1][c];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t j = L.row(q);
    if (j < d) {
      const double vq = (double)v[q];
      const double gq = gr[q] - dot * vq;
      const double vn = vq + eta * momentum_step(gq, mu, nesterov, mom, j * K + c);
      const float vf = (float)(vn * ic);
      V[j * K + c] = vf;
      if (vop) write_operand(vop, dp, dtype, scale, c, j, vf);
    }
  }
}

__global__ void k_copy_f32(const float* __restrict__ s, float* __restrict__ d, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    d[e] = s[e];
}

// Rows per thread: 8, or fewer while that leaves fewer than 256 blocks.
int update_rpt(int64_t d, int K) {
  const int64_t ng = row_groups(K);
  int rpt = kMaxRPT;
  while (rpt > 1 && cdiv(d, ng * rpt) < 256) rpt /= 2;
  return rpt;
}

template <typename F>
hipError_t dispatch_rpt(int rpt, F&& f) {
  switch (rpt) {
    case 8: return f(std::integral_constant<int, 8>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 1: return f(std::integral_constant<int, 1>{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int eigengame_blocks(int64_t d, int K) {
  return (int)cdiv(d, (int64_t)row_groups(K) * update_rpt(d, K));
}

hipError_t launch_sanger_update(float* V, const float* Z, const double* G, int64_t d, int K, int b,
                                double eta, double mu, int nesterov, float* mom, void* vop,
                                int64_t dp, int32_t dtype, const float* col_scale, int* status,
                                hipStream_t s) {
  const int rpt = update_rpt(d, K);
  const int64_t rb = (int64_t)row_groups(K) * rpt;
  const size_t lds = (size_t)K * K * sizeof(double) + (size_t)rb * K * sizeof(float);
  return dispatch_rpt(rpt, [&](auto rc) -> hipError_t {
    constexpr int RPT = decltype(rc)::value;
    hipLaunchKernelGGL(k_sanger<RPT>, dim3((unsigned)cdiv(d, rb)), dim3(kThreads), lds, s, V, Z, G,
                       d, K, b, eta, mu, nesterov, mom, vop, dp, (int)dtype, col_scale, status);
    return hipGetLastError();
  });
}

size_t eigengame_scratch_doubles(int64_t d, int K) {
  return (size_t)((int64_t)kEgSums * eigengame_blocks(d, K) * K + kEgSums * K);
}

// scratch layout: partials [nblk][6][K] | their column sums [6][K] (float64).
// vop (optional): the operand of the new V, [Kp][dp] (its padding is left as
// it is: zero from the operand built before the first step).
hipError_t launch_eigengame_update(float* V, const float* Z, const double* G, int64_t d, int K,
                                   int b, double eta, double mu, int nesterov, float* mom,
                                   double* scratch, void* vop, int64_t dp, int32_t dtype,
                                   const float* col_scale, int* status, hipStream_t s) {
  const int rpt = update_rpt(d, K);
  const int64_t rb = (int64_t)row_groups(K) * rpt;
  const int nblk = (int)cdiv(d, rb);
  double* part = scratch;
  double* sums = part + (int64_t)nblk * kEgSums * K;
  const bool two_level = nblk > kDirectPartials;
  const size_t lds = ((size_t)K * K + kThreads) * sizeof(double) + (size_t)rb * K * sizeof(float);
  const float* mom_in = mu != 0.0 ? mom : nullptr;
  return dispatch_rpt(rpt, [&](auto rc) -> hipError_t {
    constexpr int RPT = decltype(rc)::value;
    hipLaunchKernelGGL(k_eg_sums<RPT>, dim3(nblk), dim3(kThreads), lds, s, V, Z, G, d, K, b,
                       mom_in, part, status);
    if (two_level)
      hipLaunchKernelGGL(k_sum_cols, dim3(kEgSums * K), dim3(kThreads), 0, s, part, nblk,
                         kEgSums * K, sums);
    hipLaunchKernelGGL(k_eg_apply<RPT>, dim3(nblk), dim3(kThreads), lds, s, V, Z, G, d, K, b, part,
                       two_level ? (const double*)sums : nullptr, nblk, eta, mu, nesterov, mom,
                       vop, dp, (int)dtype, col_scale, status);
    return hipGetLastError();
  });
}

hipError_t launch_copy_f32(const float* src, float* dst, int64_t count, hipStream_t s) {
  int64_t g = cdiv(count, 256);
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_copy_f32, dim3(g), dim3(256), 0, s, src, dst, count);
  return hipGetLastError();
}

}  // namespace ppca
