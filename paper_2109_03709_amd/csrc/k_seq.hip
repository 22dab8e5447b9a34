// The power method's termination rule and the sequential power method
// (Sec. 2.1): one direction at a time, u <- P M u / |P M u| with M = X^T X
// (one streaming pass with K = 1) and P = I - V_<i V_<i^T the projection on
// the complement of the directions already found, until |u_t - u_{t+1}| < eps.
// These kernels work on d-vectors and a few columns of V: one workgroup,
// float64 sums in a fixed order (thread partial sums, then a tree).
#include "ppca_common.h"

namespace ppca {

namespace {

constexpr int kT = 256;

// sum over the workgroup, fixed order; every thread gets the result
__device__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// res[j] = |Vn[:, j] - Vo (Vo^T Vn[:, j])|_2, workgroup j: how far the new
// iterate's direction j lies from the previous iterate's span (Vo has
// orthonormal columns); the host takes the largest
__global__ __launch_bounds__(kT) void k_span_change(const float* __restrict__ Vn,
                                                    const float* __restrict__ Vo, int64_t d, int K,
                                                    double* __restrict__ res) {
  __shared__ double sh[kT];
  __shared__ double coef[PPCA_MAX_K];
  const int j = blockIdx.x;
  for (int i = 0; i < K; ++i) {
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < d; r += kT) s += (double)Vo[r * K + i] * (double)Vn[r * K + j];
    const double c = block_sum(s, sh);
    if (threadIdx.x == 0) coef[i] = c;
  }
  __syncthreads();
  double nn = 0.0;
  for (int64_t r = threadIdx.x; r < d; r += kT) {
    double w = (double)Vn[r * K + j];
    for (int i = 0; i < K; ++i) w -= coef[i] * (double)Vo[r * K + i];
    nn += w * w;
  }
  const double t = block_sum(nn, sh);
  if (threadIdx.x == 0) res[j] = sqrt(t);
}

// w <- w - V_<i (V_<i^T w) for column i of V (w: d-vector, float64 in LDS-free
// form: read from src, written to dst as float32 after scaling by 1 / |.|);
// returns |w| before the scaling
__device__ double project_out_normalise(const float* __restrict__ V, int64_t d, int K, int i,
                                        const float* src, float* dst, double* sh, double* coef) {
  for (int j = 0; j < i; ++j) {
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < d; r += kT) s += (double)V[r * K + j] * (double)src[r];
    const double c = block_sum(s, sh);
    if (threadIdx.x == 0) coef[j] = c;
  }
  __syncthreads();
  double nn = 0.0;
  for (int64_t r = threadIdx.x; r < d; r += kT) {
    double w = (double)src[r];
    for (int j = 0; j < i; ++j) w -= coef[j] * (double)V[r * K + j];
    nn += w * w;
  }
  const double nrm = sqrt(block_sum(nn, sh));
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int64_t r = threadIdx.x; r < d; r += kT) {
    double w = (double)src[r];
    for (int j = 0; j < i; ++j) w -= coef[j] * (double)V[r * K + j];
    dst[r] = (float)(w * inv);
  }
  __syncthreads();
  return nrm;
}

// start of direction i: u = P V[:, i] / |P V[:, i]|; state cleared
__global__ __launch_bounds__(kT) void k_seq_start(const float* __restrict__ V, int64_t d, int K,
                                                  int i, float* __restrict__ u,
                                                  SeqState* __restrict__ st, float* __restrict__ tmp,
                                                  int* status) {
  __shared__ double sh[kT];
  __shared__ double coef[PPCA_MAX_K];
  for (int64_t r = threadIdx.x; r < d; r += kT) tmp[r] = V[r * K + i];
  __syncthreads();
  const double nrm = project_out_normalise(V, d, K, i, tmp, u, sh, coef);
  if (threadIdx.x == 0) {
    st->steps = 0;
    st->done = 0;
    st->delta = 0.0;
    if (!(nrm > 0.0) || !isfinite(nrm)) set_status(status, PPCA_ERR_NOT_SPD);
  }
}

// one step of direction i from Z = M u: w = P Z / |P Z|, delta = |w - u|;
// until the direction is done: u = w, steps + 1, done when delta < eps or
// steps == max_steps (later calls of a batch change nothing)
__global__ __launch_bounds__(kT) void k_seq_step(const float* __restrict__ V, int64_t d, int K,
                                                 int i, const float* __restrict__ Z,
                                                 float* __restrict__ u, float* __restrict__ w,
                                                 SeqState* __restrict__ st, double eps,
                                                 int max_steps, int* status) {
  __shared__ double sh[kT];
  __shared__ double coef[PPCA_MAX_K];
  if (st->done) return;                 // uniform: every thread reads the same word
  const double nrm = project_out_normalise(V, d, K, i, Z, w, sh, coef);
  double dd = 0.0;
  for (int64_t r = threadIdx.x; r < d; r += kT) {
    const double df = (double)w[r] - (double)u[r];
    dd += df * df;
  }
  const double delta = sqrt(block_sum(dd, sh));
  for (int64_t r = threadIdx.x; r < d; r += kT) u[r] = w[r];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int s = st->steps + 1;
    st->steps = s;
    st->delta = delta;
    st->done = (delta < eps || s >= max_steps) ? 1 : 0;
    if (!(nrm > 0.0) || !isfinite(nrm)) {
      set_status(status, PPCA_ERR_NONFINITE);
      st->done = 1;
    }
  }
}

__global__ void k_seq_store(float* __restrict__ V, int64_t d, int K, int i,
                            const float* __restrict__ u) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < d;
       r += (int64_t)gridDim.x * blockDim.x)
    V[r * K + i] = u[r];
}

}  // namespace

hipError_t launch_span_change(const float* Vn, const float* Vo, int64_t d, int K, double* res,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_span_change, dim3(K), dim3(kT), 0, s, Vn, Vo, d, K, res);
  return hipGetLastError();
}

hipError_t launch_seq_start(const float* V, int64_t d, int K, int i, float* u, SeqState* st,
                            float* tmp, int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_seq_start, dim3(1), dim3(kT), 0, s, V, d, K, i, u, st, tmp, status);
  return hipGetLastError();
}

hipError_t launch_seq_step(const float* V, int64_t d, int K, int i, const float* Z, float* u,
                           float* w, SeqState* st, double eps, int max_steps, int* status,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_seq_step, dim3(1), dim3(kT), 0, s, V, d, K, i, Z, u, w, st, eps,
                     max_steps, status);
  return hipGetLastError();
}

hipError_t launch_seq_store(float* V, int64_t d, int K, int i, const float* u, hipStream_t s) {
  hipLaunchKernelGGL(k_seq_store, dim3((unsigned)cdiv(d, 256) < 1024 ? (unsigned)cdiv(d, 256) : 1024),
                     dim3(256), 0, s, V, d, K, i, u);
  return hipGetLastError();
}

}  // namespace ppca
