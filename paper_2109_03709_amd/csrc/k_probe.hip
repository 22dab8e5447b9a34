// Streaming-read probe: how fast one GPU reads the stored X in the access
// pattern of the streaming kernels, with no arithmetic, so that their
// achieved rates can be set against a measured ceiling as well as against the
// nominal HBM peak.
//
//   mode 0: plain 16-byte vector loads, each workgroup striding over the whole
//           matrix (row-major, ld * element bytes per row);
//   mode 1: the LDS-DMA pipeline of the power-pass kernels: a workgroup takes
//           a tile of 32 KB / SEG rows and walks across it SEG bytes of every
//           row per step (global_load_lds_dwordx4 into three 32 KB LDS
//           stages, two in flight), SEG = 128, 256 or 512.  The bytes in
//           flight per CU are those of k_xvy; only the row segment changes.
//
// Every 16-byte chunk of rows [0, n) x bytes [0, ld * es) is read exactly once
// and XOR-folded into sink[workgroup] (so the loads cannot be dropped, and a
// test can check that the whole matrix was read once).
#include "lds_dma.h"

namespace ppca {

using dma::dma16;
using dma::raw_barrier;
using dma::wait_lgkm0;
using dma::wait_vmcnt;

namespace {

constexpr int kProbeStage = 32 * 1024;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_probe_vec(const uint8_t* __restrict__ x, int64_t n,
                                                   int64_t row_bytes, uint32_t* __restrict__ sink) {
  const int64_t chunks_per_row = row_bytes / 16;
  const int64_t total = n * chunks_per_row;
  u32x4 acc = {0u, 0u, 0u, 0u};
  const u32x4* p = reinterpret_cast<const u32x4*>(x);
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // four loads in flight per thread
  for (; e + 3 * stride < total; e += 4 * stride) {
    u32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(p + e + u * stride);
#pragma unroll
    for (int u = 0; u < 4; ++u) acc ^= v[u];
  }
  for (; e < total; e += stride) acc ^= __builtin_nontemporal_load(p + e);
  uint32_t a = acc.x ^ acc.y ^ acc.z ^ acc.w;
  __shared__ uint32_t red[256];
  red[threadIdx.x] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int i = 0; i < 256; ++i) s ^= red[i];
    sink[blockIdx.x] = s;
  }
}

// SEG bytes of a row per step; a stage holds RT = 32 KB / SEG rows.  DMA j
// of wave w covers rows RPD * (w * DI + j) .. + RPD - 1 (RPD = 1024 / SEG rows
// per 1 KB DMA), lane -> (row lane / CPR, chunk lane % CPR), CPR = SEG / 16.
// Tiles past n and segments past row_bytes are not read: a lane whose chunk
// lies outside the matrix loads the matrix's first chunk instead and leaves
// it out of the fold.
template <int SEG>
__global__ __launch_bounds__(256, 1) void k_probe_dma(const uint8_t* __restrict__ x, int64_t n,
                                                      int64_t row_bytes,
                                                      uint32_t* __restrict__ sink) {
  constexpr int RT = kProbeStage / SEG, CPR = SEG / 16, RPD = 64 / CPR;
  constexpr int DI = kProbeStage / 1024 / 4;   // DMAs per wave per step
  static_assert(2 * DI < 64, "vmcnt range");
  __shared__ __attribute__((aligned(16))) uint8_t st[3 * kProbeStage];
  const int t = threadIdx.x, lane = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int64_t ntile = (n + RT - 1) / RT;
  const int64_t mytiles = ntile > blockIdx.x ? (ntile - 1 - blockIdx.x) / gridDim.x + 1 : 0;
  const int64_t nk = (row_bytes + SEG - 1) / SEG;
  const int64_t nsteps = mytiles * nk;
  uint32_t fold = 0;
  if (nsteps > 0) {
    // issue side: step iss = (tile ordinal, segment ik); past the last step the
    // last one is loaded again (every wave issues the same count) and not folded
    int64_t iss = 0, ik = 0, itile = 0;
    auto chunk_of = [&](int64_t tord, int64_t seg, int j, int64_t& off) -> bool {
      const int64_t row = ((int64_t)blockIdx.x + tord * gridDim.x) * RT + RPD * (w * DI + j) +
                          lane / CPR;
      const int64_t col = seg * SEG + (int64_t)(lane % CPR) * 16;
      const bool in = row < n && col + 16 <= row_bytes;
      off = in ? row * row_bytes + col : 0;
      return in;
    };
    auto issue = [&](int b) __attribute__((always_inline)) {
      uint8_t* sb = st + b * kProbeStage;
#pragma unroll
      for (int j = 0; j < DI; ++j) {
        int64_t off;
        chunk_of(itile, ik, j, off);
        dma16(x + off, sb + (w * DI + j) * 1024);
      }
      if (iss < nsteps) {
        ++iss;
        if (iss < nsteps && ++ik == nk) {
          ik = 0;
          ++itile;
        }
      }
    };
    issue(0);
    issue(1);
    int b = 0;
    int64_t ctile = 0, cseg = 0;
    for (int64_t s = 0; s < nsteps; ++s) {
      wait_vmcnt<DI>();                    // this wave's DMA of step s has landed
      raw_barrier();                       // ... and every wave's; stage (b+2)%3 is free
      issue(b == 0 ? 2 : b - 1);
      // fold this wave's own chunks of the step (read back from LDS)
      const uint8_t* sb = st + b * kProbeStage;
#pragma unroll
      for (int j = 0; j < DI; ++j) {
        int64_t off;
        if (chunk_of(ctile, cseg, j, off)) {
          const uint4 v = *reinterpret_cast<const uint4*>(sb + (w * DI + j) * 1024 + lane * 16);
          fold ^= v.x ^ v.y ^ v.z ^ v.w;
        }
      }
      wait_lgkm0();
      if (++cseg == nk) {
        cseg = 0;
        ++ctile;
      }
      b = b == 2 ? 0 : b + 1;
    }
    wait_vmcnt<0>();
  }
  __shared__ uint32_t red[256];
  __syncthreads();
  red[t] = fold;
  __syncthreads();
  if (t == 0) {
    uint32_t s = 0;
    for (int i = 0; i < 256; ++i) s ^= red[i];
    sink[blockIdx.x] = s;
  }
}

}  // namespace

int probe_grid(int32_t mode) { return mode == 0 ? 4 * kNumCU : kNumCU; }

hipError_t launch_read_probe(const void* x, int64_t n, int64_t row_bytes, int32_t mode,
                             int32_t seg, uint32_t* sink, hipStream_t s) {
  const uint8_t* p = static_cast<const uint8_t*>(x);
  if (mode == 0) {
    hipLaunchKernelGGL(k_probe_vec, dim3(probe_grid(0)), dim3(256), 0, s, p, n, row_bytes, sink);
  } else if (seg == 128) {
    hipLaunchKernelGGL(k_probe_dma<128>, dim3(probe_grid(1)), dim3(256), 0, s, p, n, row_bytes,
                       sink);
  } else if (seg == 256) {
    hipLaunchKernelGGL(k_probe_dma<256>, dim3(probe_grid(1)), dim3(256), 0, s, p, n, row_bytes,
                       sink);
  } else if (seg == 512) {
    hipLaunchKernelGGL(k_probe_dma<512>, dim3(probe_grid(1)), dim3(256), 0, s, p, n, row_bytes,
                       sink);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ppca
