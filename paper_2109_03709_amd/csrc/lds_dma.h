// Device helpers of the LDS-DMA software pipelines (k_stream.hip, k_group.hip):
// explicit vmcnt / lgkmcnt waits, a workgroup barrier without the memory
// fence of __syncthreads, and one global_load_lds_dwordx4 per call.
#pragma once
#include "ppca_common.h"

namespace ppca {
namespace dma {

__device__ inline bf16x8_t as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8_t, v); }

// s_waitcnt with vmcnt = N (expcnt and lgkmcnt left unconstrained)
template <int N>
__device__ __attribute__((always_inline)) inline void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}
__device__ __attribute__((always_inline)) inline void wait_lgkm0() {
  __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (0 << 8) | (3 << 14));
}
// workgroup barrier without the memory fence of __syncthreads (which would
// wait for every outstanding DMA); the signal fences keep the compiler from
// moving LDS accesses across it
__device__ __attribute__((always_inline)) inline void raw_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_sched_barrier(0);
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_sched_barrier(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
// One global_load_lds_dwordx4: lane i's 16 bytes at g go to LDS byte
// lds + 16 i; `lds` must be the same for the whole wavefront.  Written as
// inline asm so that the compiler's wait insertion, which cannot tell the
// three stages apart and would make every LDS read wait for every DMA in
// flight, does not see it: the kernel places its own waits (wait_vmcnt before
// each barrier).  The instruction has no register result; M0 carries the LDS
// base and is set in the same block (nothing else in these kernels uses M0).
__device__ __attribute__((always_inline)) inline void dma16(const void* g, void* lds) {
  const uint32_t base = __builtin_amdgcn_readfirstlane(
      (uint32_t)(uintptr_t)(__attribute__((address_space(3))) void*)lds);
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
               :
               : "v"(g), "s"(base)
               : "memory");
}

// The same with the address split into a wavefront-uniform base (SGPR pair)
// and a 32-bit per-lane byte offset: lane i's 16 bytes at sbase + voff go to
// LDS byte lds + 16 i.  Saves the 64-bit address arithmetic per lane.
__device__ __attribute__((always_inline)) inline void dma16s(const void* sbase, uint32_t voff,
                                                             void* lds) {
  const uint32_t base = __builtin_amdgcn_readfirstlane(
      (uint32_t)(uintptr_t)(__attribute__((address_space(3))) void*)lds);
  // readfirstlane returns a signed int: each half goes through uint32_t so
  // that widening zero-extends it
  const uint64_t a = (uint64_t)(uintptr_t)sbase;
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint64_t sa = ((uint64_t)hi << 32) | (uint64_t)lo;
  asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, %1"
               :
               : "v"(voff), "s"(sa), "s"(base)
               : "memory");
}

}  // namespace dma
}  // namespace ppca
