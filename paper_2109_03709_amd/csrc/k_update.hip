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

constexpr int kRowsPerBlock = 16;

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

__global__ __launch_bounds__(256) void k_sanger(float* __restrict__ V, const float* __restrict__ Z,
                                                const double* __restrict__ G, int64_t d, int K,
                                                int b, double eta, double mu, int nesterov,
                                                float* __restrict__ mom, int* status) {
  __shared__ double Gs[kMaxK * kMaxK];
  __shared__ double Vs[kRowsPerBlock * kMaxK];
  if (status_set(status)) return;
  const int64_t j0 = (int64_t)blockIdx.x * kRowsPerBlock;
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
    const int i = e / K, c = e % K;
    Gs[e] = i <= c ? G[e] : 0.0;
  }
  for (int e = threadIdx.x; e < kRowsPerBlock * K; e += blockDim.x) {
    const int64_t j = j0 + e / K;
    Vs[e] = j < d ? (double)V[j * K + e % K] : 0.0;
  }
  __syncthreads();
  const double inv_b = 1.0 / (double)b;
  for (int e = threadIdx.x; e < kRowsPerBlock * K; e += blockDim.x) {
    const int r = e / K, c = e % K;
    const int64_t j = j0 + r;
    if (j >= d) continue;
    double s = (double)Z[j * K + c];
    for (int i = 0; i <= c; ++i) s = fma(-Vs[r * K + i], Gs[i * K + c], s);
    const double step = momentum_step(s * inv_b, mu, nesterov, mom, j * K + c);
    V[j * K + c] = (float)(Vs[r * K + c] + eta * step);
  }
}

// EigenGame, phase 1: grad = (2/b) Z R, per-block partial dots v_c . grad_c.
__global__ __launch_bounds__(256) void k_eg_grad(const float* __restrict__ V,
                                                 const float* __restrict__ Z,
                                                 const double* __restrict__ G, int64_t d, int K,
                                                 int b, double* __restrict__ grad,
                                                 double* __restrict__ pdot, int* status) {
  __shared__ double Rs[kMaxK * kMaxK];
  __shared__ double Zs[kRowsPerBlock * kMaxK];
  __shared__ double red[kRowsPerBlock * kMaxK];
  if (status_set(status)) return;
  const int64_t j0 = (int64_t)blockIdx.x * kRowsPerBlock;
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
    const int i = e / K, c = e % K;
    double r = 0.0;
    if (i == c) r = 1.0;
    else if (i < c && G[i * K + i] > 1e-300) r = -G[e] / G[i * K + i];
    Rs[e] = r;
  }
  for (int e = threadIdx.x; e < kRowsPerBlock * K; e += blockDim.x) {
    const int64_t j = j0 + e / K;
    Zs[e] = j < d ? (double)Z[j * K + e % K] : 0.0;
  }
  __syncthreads();
  const double sc = 2.0 / (double)b;
  for (int e = threadIdx.x; e < kRowsPerBlock * K; e += blockDim.x) {
    const int r = e / K, c = e % K;
    const int64_t j = j0 + r;
    double gv = 0.0;
    if (j < d) {
      double s = 0.0;
      for (int i = 0; i <= c; ++i) s = fma(Zs[r * K + i], Rs[i * K + c], s);
      gv = sc * s;
      grad[j * K + c] = gv;
      red[e] = (double)V[j * K + c] * gv;
    } else {
      red[e] = 0.0;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < K; c += blockDim.x) {
    double s = 0.0;
    for (int r = 0; r < kRowsPerBlock; ++r) s += red[r * K + c];
    pdot[(int64_t)blockIdx.x * K + c] = s;
  }
}

// EigenGame, phase 2: Riemannian projection, momentum, ascent step; partial norms.
__global__ __launch_bounds__(256) void k_eg_step(const float* __restrict__ V,
                                                 const double* __restrict__ grad,
                                                 const double* __restrict__ pdot, int nblk,
                                                 int64_t d, int K, double eta, double mu,
                                                 int nesterov, float* __restrict__ mom,
                                                 double* __restrict__ vnew,
                                                 double* __restrict__ pnorm, int* status) {
  __shared__ double dots[kMaxK];
  __shared__ double red[kRowsPerBlock * kMaxK];
  if (status_set(status)) return;
  for (int c = threadIdx.x; c < K; c += blockDim.x) {
    double s = 0.0;
    for (int w = 0; w < nblk; ++w) s += pdot[(int64_t)w * K + c];
    dots[c] = s;
  }
  __syncthreads();
  const int64_t j0 = (int64_t)blockIdx.x * kRowsPerBlock;
  for (int e = threadIdx.x; e < kRowsPerBlock * K; e += blockDim.x) {
    const int r = e / K, c = e % K;
    const int64_t j = j0 + r;
    double sq = 0.0;
    if (j < d) {
      const double v = (double)V[j * K + c];
      const double g = grad[j * K + c] - dots[c] * v;
      const double step = momentum_step(g, mu, nesterov, mom, j * K + c);
      const double vn = v + eta * step;
      vnew[j * K + c] = vn;
      sq = vn * vn;
    }
    red[e] = sq;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < K; c += blockDim.x) {
    double s = 0.0;
    for (int r = 0; r < kRowsPerBlock; ++r) s += red[r * K + c];
    pnorm[(int64_t)blockIdx.x * K + c] = s;
  }
}

// EigenGame, phase 3: unit-norm columns.
__global__ __launch_bounds__(256) void k_eg_normalise(float* __restrict__ V,
                                                      const double* __restrict__ vnew,
                                                      const double* __restrict__ pnorm, int nblk,
                                                      int64_t d, int K, int* status) {
  __shared__ double inv[kMaxK];
  if (status_set(status)) return;
  for (int c = threadIdx.x; c < K; c += blockDim.x) {
    double s = 0.0;
    for (int w = 0; w < nblk; ++w) s += pnorm[(int64_t)w * K + c];
    inv[c] = 1.0 / sqrt(s);
    if (!(s > 0.0) || !isfinite(s)) set_status(status, PPCA_ERR_NONFINITE);
  }
  __syncthreads();
  const int64_t j0 = (int64_t)blockIdx.x * kRowsPerBlock;
  for (int e = threadIdx.x; e < kRowsPerBlock * K; e += blockDim.x) {
    const int64_t j = j0 + e / K;
    const int c = e % K;
    if (j < d) V[j * K + c] = (float)(vnew[j * K + c] * inv[c]);
  }
}

__global__ void k_copy_f32(const float* __restrict__ s, float* __restrict__ d, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    d[e] = s[e];
}

}  // namespace

hipError_t launch_sanger_update(float* V, const float* Z, const double* G, int64_t d, int K, int b,
                                double eta, double mu, int nesterov, float* mom, int* status,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_sanger, dim3((unsigned)cdiv(d, kRowsPerBlock)), dim3(256), 0, s, V, Z, G, d,
                     K, b, eta, mu, nesterov, mom, status);
  return hipGetLastError();
}

// scratch layout: grad [d*K] | vnew [d*K] | pdot [nblk*K] | pnorm [nblk*K]   (float64)
hipError_t launch_eigengame_update(float* V, const float* Z, const double* G, int64_t d, int K,
                                   int b, double eta, double mu, int nesterov, float* mom,
                                   double* scratch, int* status, hipStream_t s) {
  const int nblk = (int)cdiv(d, kRowsPerBlock);
  double* grad = scratch;
  double* vnew = grad + d * K;
  double* pdot = vnew + d * K;
  double* pnorm = pdot + (int64_t)nblk * K;
  hipLaunchKernelGGL(k_eg_grad, dim3(nblk), dim3(256), 0, s, V, Z, G, d, K, b, grad, pdot, status);
  hipLaunchKernelGGL(k_eg_step, dim3(nblk), dim3(256), 0, s, V, grad, pdot, nblk, d, K, eta, mu,
                     nesterov, mom, vnew, pnorm, status);
  hipLaunchKernelGGL(k_eg_normalise, dim3(nblk), dim3(256), 0, s, V, vnew, pnorm, nblk, d, K,
                     status);
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
