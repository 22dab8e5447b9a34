// Data preparation: centring (the paper works with a centred dataset, Sec. 1)
// and conversion to the storage type of the streaming passes.
//
//   mu_j = (sum_r x_rj) / n   -- double-double column sums, rounded once
//   c_rj = float32(double(x_rj) - mu_j)
//   f32 : c           bf16 : nearest bf16 of c (ties to even)
//   fp8 : nearest e4m3 of float32(c_rj / s_j), ties to even, saturating at 448,
//         s_j = float32(max_r |c_rj| / 448)  (1 for an all-zero column)
#include "ppca_common.h"

namespace ppca {

namespace {

constexpr int kPrepRows = 4096;   // rows per block of the column reductions

__device__ inline void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__device__ inline float centred(float x, double mu) { return (float)((double)x - mu); }

// fp8 e4m3 ("fn": bias 7, max 448) code of a finite float: round to nearest,
// ties to even, saturate.  Subnormals are multiples of 2^-9.
__device__ inline uint32_t e4m3_encode(float v) {
  const uint32_t sign = (__float_as_uint(v) >> 24) & 0x80u;
  const float a = fabsf(v);
  uint32_t mag;
  if (!(a < 448.0f)) {
    mag = 0x7Eu;
  } else if (a < 0.015625f) {
    mag = (uint32_t)rintf(a * 512.0f);            // 0..8; 8 is the smallest normal
  } else {
    int e;
    const float m = frexpf(a, &e);                // a = m 2^e, m in [0.5, 1)
    int E = e - 1;                                // a = (2m) 2^E, 2m in [1, 2)
    uint32_t q = (uint32_t)rintf((2.0f * m - 1.0f) * 8.0f);
    if (q == 8u) { q = 0u; E += 1; }
    mag = ((uint32_t)(E + 7) << 3) | q;
  }
  return sign | mag;
}

__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ x, int64_t n, int64_t d,
                                                int64_t ld, double* __restrict__ part) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d) return;
  const int64_t r0 = (int64_t)blockIdx.y * kPrepRows;
  const int64_t r1 = r0 + kPrepRows < n ? r0 + kPrepRows : n;
  double hi = 0.0, lo = 0.0;
  auto add = [&](float v) {
    double s, e;
    two_sum(hi, (double)v, s, e);
    hi = s;
    lo += e;
  };
  // rows in order; eight loads in flight ahead of the dependent sums
  int64_t r = r0;
  for (; r + 8 <= r1; r += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = x[(r + u) * ld + j];
#pragma unroll
    for (int u = 0; u < 8; ++u) add(v[u]);
  }
  for (; r < r1; ++r) add(x[r * ld + j]);
  double s, e;
  two_sum(hi, lo, s, e);
  part[((int64_t)blockIdx.y * d + j) * 2 + 0] = s;
  part[((int64_t)blockIdx.y * d + j) * 2 + 1] = e;
}

__global__ __launch_bounds__(256) void k_colmean(const double* __restrict__ part, int nrb,
                                                 int64_t n, int64_t d, double* __restrict__ mean,
                                                 double* __restrict__ mean_out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d) return;
  double hi = 0.0, lo = 0.0;
  for (int b = 0; b < nrb; ++b) {
    double s, e;
    two_sum(hi, part[((int64_t)b * d + j) * 2 + 0], s, e);
    hi = s;
    lo += e + part[((int64_t)b * d + j) * 2 + 1];
  }
  double s, e;
  two_sum(hi, lo, s, e);            // s = correctly rounded value of hi + lo
  const double mu = s / (double)n;
  mean[j] = mu;
  if (mean_out) mean_out[j] = mu;
}

__global__ __launch_bounds__(256) void k_colmax(const float* __restrict__ x, int64_t n, int64_t d,
                                                int64_t ld, const double* __restrict__ mean,
                                                float* __restrict__ part) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d) return;
  const int64_t r0 = (int64_t)blockIdx.y * kPrepRows;
  const int64_t r1 = r0 + kPrepRows < n ? r0 + kPrepRows : n;
  const double mu = mean[j];
  float m = 0.f;
  int64_t r = r0;
  for (; r + 8 <= r1; r += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = x[(r + u) * ld + j];
#pragma unroll
    for (int u = 0; u < 8; ++u) m = fmaxf(m, fabsf(centred(v[u], mu)));
  }
  for (; r < r1; ++r) m = fmaxf(m, fabsf(centred(x[r * ld + j], mu)));
  part[(int64_t)blockIdx.y * d + j] = m;
}

__global__ __launch_bounds__(256) void k_colscale(const float* __restrict__ part, int nrb,
                                                  int64_t d, float* __restrict__ scale) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d) return;
  float m = 0.f;
  for (int b = 0; b < nrb; ++b) m = fmaxf(m, part[(int64_t)b * d + j]);
  scale[j] = m > 0.f ? __fdiv_rn(m, 448.0f) : 1.0f;
}

template <int OUT>
__global__ __launch_bounds__(256) void k_quantize(const float* __restrict__ x, int64_t n, int64_t d,
                                                  int64_t ldx, const double* __restrict__ mean,
                                                  const float* __restrict__ scale,
                                                  void* __restrict__ out, int64_t ldo) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d) return;
  const double mu = mean[j];
  const float s = OUT == PPCA_FP8_E4M3 ? scale[j] : 1.0f;
  for (int64_t r = blockIdx.y; r < n; r += gridDim.y) {
    const float c = centred(x[r * ldx + j], mu);
    if (OUT == PPCA_F32) {
      reinterpret_cast<float*>(out)[r * ldo + j] = c;
    } else if (OUT == PPCA_BF16) {
      reinterpret_cast<uint16_t*>(out)[r * ldo + j] = (uint16_t)f32_to_bf16_bits(c);
    } else {
      reinterpret_cast<uint8_t*>(out)[r * ldo + j] = (uint8_t)e4m3_encode(__fdiv_rn(c, s));
    }
  }
}

}  // namespace

int prep_row_blocks(int64_t n) { return (int)cdiv(n, kPrepRows); }

hipError_t launch_center_quantize(const float* x, int64_t n, int64_t d, int64_t ldx,
                                  int32_t out_dtype, void* out, int64_t ldo, float* col_scale,
                                  double* mean_out, double* ws_sums, float* ws_max,
                                  double* ws_mean, hipStream_t s) {
  const int nrb = prep_row_blocks(n);
  const dim3 cgrid((unsigned)cdiv(d, 256), (unsigned)nrb);
  const dim3 c1((unsigned)cdiv(d, 256));
  hipLaunchKernelGGL(k_colsum, cgrid, dim3(256), 0, s, x, n, d, ldx, ws_sums);
  hipLaunchKernelGGL(k_colmean, c1, dim3(256), 0, s, ws_sums, nrb, n, d, ws_mean, mean_out);
  if (out_dtype == PPCA_FP8_E4M3) {
    hipLaunchKernelGGL(k_colmax, cgrid, dim3(256), 0, s, x, n, d, ldx, ws_mean, ws_max);
    hipLaunchKernelGGL(k_colscale, c1, dim3(256), 0, s, ws_max, nrb, d, col_scale);
  }
  int64_t gy = n < 8192 ? n : 8192;
  const dim3 qgrid((unsigned)cdiv(d, 256), (unsigned)gy);
  if (out_dtype == PPCA_F32)
    hipLaunchKernelGGL(k_quantize<PPCA_F32>, qgrid, dim3(256), 0, s, x, n, d, ldx, ws_mean,
                       col_scale, out, ldo);
  else if (out_dtype == PPCA_BF16)
    hipLaunchKernelGGL(k_quantize<PPCA_BF16>, qgrid, dim3(256), 0, s, x, n, d, ldx, ws_mean,
                       col_scale, out, ldo);
  else
    hipLaunchKernelGGL(k_quantize<PPCA_FP8_E4M3>, qgrid, dim3(256), 0, s, x, n, d, ldx, ws_mean,
                       col_scale, out, ldo);
  return hipGetLastError();
}

}  // namespace ppca
