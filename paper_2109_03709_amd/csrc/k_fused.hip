// Single-read power pass for bf16 data (block power step, Sec. 2.1):
// Z = X^T bf16(X V') with every element of X read from HBM once.
//
// Y = X V' reduces over the columns of X and Z = X^T Y over its rows, and at
// d x Kp = 2048 x 128 the float32 Z (1 MB) does not fit one CU.  So the 256
// workgroups (one per CU, all resident: cooperative launch) form clusters of
// C workgroups on one XCD; member m of a cluster owns the 256 columns
// [256 m, 256 m + 256) of X and keeps that slice of Z in its accumulators.
// Clusters are formed at run time from the XCD each workgroup finds itself
// on (hardware register XCC_ID and a ticket counter per XCD): the L2s of
// different XCDs are not coherent for the loads used here, and the order in
// which workgroups are dealt to XCDs changes from launch to launch.
// A cluster walks its row tiles (32 rows each) in a software pipeline; in
// iteration q a member
//   - computes Y_m(q) = X(q)[:, slice m] V'[slice m, :], a 32 x Kp float32
//     partial, and stores it to the cluster's exchange slot;
//   - sums one column block (Kp / C columns) of the C partials of tile q-2 in
//     member order, rounds it to bf16 and stores it (reduce-scatter);
//   - copies the whole bf16 tile q-5 back into LDS (all-gather);
//   - adds Z_m += X(q-6)[:, slice m]^T Y(q-6), from the X tile kept in LDS;
//   - then posts iteration q in its progress word (q + 1, a plain store),
//     once its partial of tile q and its slice of tile q-3 are known to be
//     complete (both precede loads that have returned).
// Each iteration waits until every member has posted iteration q-2, which
// they did a whole iteration earlier: the wait normally succeeds at its first
// read, and it covers both the partials of tile q-2 and the slices of tile
// q-5.  Partials, slices and progress words stay in the XCD's L2: stores are
// written through the CU's L1, and loads of another member's data use sc1
// (device scope: they skip the L1, which may hold a stale line of the same
// address).  Every wait is bounded; an expired wait or a workgroup that
// cannot join a cluster ends the pass with a status code instead of a hang.
//
// Arithmetic: Y(p) = bf16(sum over members, in member order, of the float32
// partials of 256-column slices) -- the same bf16 operand the two-kernel pass
// rounds, summed in a different order; Z partials per (slice, cluster) are
// summed in float64 in a fixed order by the stream reduction, so results are
// bitwise reproducible run to run.
//
// Layouts (workspace):
//   ex    [cluster][slot][member][Kp][32] float32  Y partials (column major)
//   ybg   [cluster][slot][4][Kp][8] bf16           rounded Y tile, the blocked
//                                                  layout of the Z product's B
//   flags [cluster] progress words (C ints in one 128-byte line), then 8 XCD
//         ticket counters and the abort word, 128 bytes apart; zeroed before
//         every launch
//   part  [member = 256-column tile][cluster = split][Kp][256] float32
#include "lds_dma.h"

namespace ppca {

namespace {

using namespace dma;

constexpr int FR = 32;            // rows per tile
constexpr int FSW = 256;          // columns of X per member
constexpr int FXB = 8;            // X tile buffers in LDS (tiles q-6 .. q+1)
constexpr int FSLOT = 8;          // exchange slots per cluster
constexpr int FFLAG = 32;         // ints per flag (one 128-byte line)
constexpr int FXD = 4;            // X DMAs per wave per tile (16 KB / 4 waves / 1 KB)

__device__ inline unsigned xcc_id() {
  unsigned v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
  return v & 0xFu;
}

// global_load_lds_dwordx4 at device scope (sc1): skips the CU's L1, so a line
// of the same exchange slot cached by an earlier use is not returned
__device__ __attribute__((always_inline)) inline void dma16_sc1(const void* g, void* lds) {
  const uint32_t base = __builtin_amdgcn_readfirstlane(
      (uint32_t)(uintptr_t)(__attribute__((address_space(3))) void*)lds);
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off sc1"
               :
               : "v"(g), "s"(base)
               : "memory");
}

__device__ inline uint4 and4f(uint4 a, uint4 m) {
  return make_uint4(a.x & m.x, a.y & m.y, a.z & m.z, a.w & m.w);
}

// mask of the bf16 elements of a 16-byte chunk starting at column col that lie below d
__device__ inline uint4 tail_mask(int64_t col, int64_t d) {
  int64_t nv = d - col;
  nv = nv < 0 ? 0 : (nv > 8 ? 8 : nv);
  const int v = (int)nv * 2;
  uint32_t w[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int b = v - 4 * i;
    w[i] = b >= 4 ? 0xFFFFFFFFu : (b <= 0 ? 0u : 0x0000FFFFu);
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// Bounded wait, by one whole wavefront, until the progress word of every
// member (lane l < C reads member l's word with a device-scope load, i.e. from
// the XCD's L2) is at least `want`.  Returns false when the abort word is set
// or the spin limit is reached (then sets the abort word).
template <int C>
__device__ inline bool wait_members(const int* words, int want, int* abort_word, int spin_limit) {
  const int lane = threadIdx.x & 63;
  for (int spins = 0;; ++spins) {
    const int v = lane < C ? __hip_atomic_load(words + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                           : want;
    if (__all(v >= want)) return true;
    if (__hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
        spins >= spin_limit) {
      if (lane == 0) __hip_atomic_store(abort_word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

template <int NB2, int C>
__global__ __launch_bounds__(256, 1) void k_xxv(const uint8_t* x, int64_t n, int64_t d, int64_t ld,
                                                int64_t rstart, int64_t rows, const uint8_t* vop,
                                                int64_t dp, float* ex, uint16_t* ybg, int* flags,
                                                float* dummy, float* part, int* status,
                                                int spin_limit) {
  constexpr int Kp = 32 * NB2;
  constexpr int NCL = 256 / C;                   // clusters
  constexpr int CPX = 32 / C;                    // clusters per XCD
  constexpr int KPC = Kp / C;                    // Y columns each member reduces
  constexpr int ITEMS = KPC * 8;                 // (column, 4-row group) items per member
  constexpr int RIT = (ITEMS + 255) / 256;       // items per thread
  constexpr int YTB = 4 * Kp * 16;               // bytes of a bf16 Y tile
  constexpr int YDPW = (YTB + 4095) / 4096;      // Y-tile DMAs per wave
  constexpr int YSB = 4096 * YDPW;               // LDS bytes of a Y-tile slot
  constexpr int XTB = FR * FSW * 2;              // bytes of an X tile slice (16 KB)
  // VMEM operations of one wave per iteration, in issue order
  constexpr int YS = 4;                          // Y partial stores
  constexpr int RL = C * RIT;                    // partial loads of the reduction
  constexpr int YSS = RIT;                       // bf16 slice stores
  // waits, as "at most N younger operations outstanding" (operations issued
  // by wave 0 alone -- flag loads and atomics -- only make them stricter)
  constexpr int W_X = YS + RL + YDPW + YSS + FXD;     // X tile q (issued two iterations back)
  constexpr int W_Y = YSS + FXD + YS + RL + YDPW;     // Y tile q-6 (issued last iteration)
  constexpr int W_R = YDPW;                           // reduction loads of this iteration
  static_assert(Kp % C == 0 && KPC >= 1, "column blocks");
  static_assert(W_X < 64 && W_Y < 64, "vmcnt range");

  __shared__ __attribute__((aligned(16))) uint8_t xs[FXB * XTB];
  __shared__ __attribute__((aligned(16))) uint8_t ys[2 * YSB];
  __shared__ int s_ctl[3];   // abort, cluster, member

  const int t = threadIdx.x, lane = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int l32 = lane & 31, hl = lane >> 5;
  int* abort_word = flags + (NCL + 8) * FFLAG;
  // cluster and member from the XCD this workgroup runs on: the i-th
  // workgroup to arrive on XCD x is member i % C of cluster x * CPX + i / C
  if (t == 0) {
    const unsigned xcc = xcc_id();
    int ok = xcc < 8u;
    int tk = 0;
    if (ok) {
      tk = __hip_atomic_fetch_add(flags + (NCL + (int)xcc) * FFLAG, 1, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
      ok = tk < 32;
    }
    if (!ok) {
      set_status(status, PPCA_ERR_PLACEMENT);
      __hip_atomic_store(abort_word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    s_ctl[0] = ok ? 0 : 1;
    s_ctl[1] = ok ? (int)xcc * CPX + tk / C : 0;
    s_ctl[2] = ok ? tk % C : 0;
  }
  __syncthreads();
  const int cl = __builtin_amdgcn_readfirstlane(s_ctl[1]);
  const int m = __builtin_amdgcn_readfirstlane(s_ctl[2]);
  const int64_t ntile = (rows + FR - 1) / FR;
  const int64_t T = cl < ntile ? (ntile - 1 - cl) / NCL + 1 : 0;   // tiles of this cluster
  const int64_t col0 = (int64_t)m * FSW;

  // ---- operand V'^T [Kp][dp] of this member's slice, wave w < NB2: N block w
  uint4 vf[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int64_t col = col0 + 16 * s + 8 * hl;
    vf[s] = make_uint4(0u, 0u, 0u, 0u);
    if (w < NB2 && col < dp)
      vf[s] = *reinterpret_cast<const uint4*>(vop + ((int64_t)(32 * w + l32) * dp + col) * 2);
  }

  // ---- X DMA sources: DMA jj of wave w fills LDS rows 2 (4 w + jj) + lane / 32
  // of a tile, slot lane % 32 holding chunk (lane % 32) ^ (row & 7)
  int64_t xcol[FXD];
  uint32_t tailbits = 0;
#pragma unroll
  for (int jj = 0; jj < FXD; ++jj) {
    const int rr = 2 * (4 * w + jj) + (lane >> 5);
    const int gc = (lane & 31) ^ (rr & 7);
    const int64_t col = col0 + 8 * gc;
    xcol[jj] = col < d ? col : 0;
    if (col < d && col + 8 > d) tailbits |= 1u << jj;
  }
  auto tile_row0 = [&](int64_t p) -> int64_t {   // first pass row of cluster tile p
    const int64_t pc = p < T ? p : T - 1;
    return (cl + pc * NCL) * FR;
  };
  auto issue_x = [&](int64_t p) __attribute__((always_inline)) {
    uint8_t* dst = xs + (int)(p % FXB) * XTB;
    const int64_t r0 = tile_row0(p);
#pragma unroll
    for (int jj = 0; jj < FXD; ++jj) {
      const int rr = 2 * (4 * w + jj) + (lane >> 5);
      int64_t i = r0 + rr;
      if (i >= rows) i = rows - 1;                 // rows past the pass: any valid row
      int64_t r = rstart + i;
      if (r >= n) r %= n;
      dma16(x + (r * ld + xcol[jj]) * 2, dst + (4 * w + jj) * 1024);
    }
  };
  auto fix_tail = [&](int64_t p) __attribute__((always_inline)) {
    uint8_t* src = xs + (int)(p % FXB) * XTB;
#pragma unroll
    for (int jj = 0; jj < FXD; ++jj)
      if (tailbits & (1u << jj)) {
        uint4* slot = reinterpret_cast<uint4*>(src + (4 * w + jj) * 1024 + lane * 16);
        *slot = and4f(*slot, tail_mask(xcol[jj], d));
      }
  };

  // exchange addresses
  auto ex_slot = [&](int64_t p, int mm) -> float* {
    return ex + (((int64_t)cl * FSLOT + (int)(p % FSLOT)) * C + mm) * (Kp * FR);
  };
  auto yb_slot = [&](int64_t p) -> uint16_t* {
    return ybg + ((int64_t)cl * FSLOT + (int)(p % FSLOT)) * (YTB / 2);
  };
  // progress words of the cluster (one 128-byte line): member m writes p + 1
  // once every store it made up to and including the partial of tile p (and
  // the bf16 slice of tile p - 3) is complete
  int* words = flags + (int64_t)cl * FFLAG;
  const __amdgpu_buffer_rsrc_t exr = __builtin_amdgcn_make_buffer_rsrc(
      (void*)ex, 0, (int)((int64_t)NCL * FSLOT * C * Kp * FR * 4), 0x00020000);

  f32x16_t zacc[2][NB2];
#pragma unroll
  for (int v = 0; v < 2; ++v)
#pragma unroll
    for (int nb = 0; nb < NB2; ++nb) zacc[v][nb] = f32x16_t{};

  const bool live = s_ctl[0] == 0 && T > 0;
  if (live) {
    issue_x(0);
    issue_x(1);
  }
  // iteration q: Y(q); reduction of tile q-2; bf16 tile q-5 -> LDS; Z(q-6)
  const int64_t niter = live ? T + 6 : 0;
  for (int64_t q = 0; q < niter; ++q) {
    // (0) wave 0 starts reading the progress words (iteration q-2 was posted a
    // whole iteration ago); they are needed at (3)
    const int want = (int)(q - 1);
    int seen = want;
    if (w == 0 && q >= 2 && lane < C)
      seen = __hip_atomic_load(words + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // (1) X tile q has landed in every wave
    if (q < 2) wait_vmcnt<0>();
    else wait_vmcnt<W_X>();
    if (tailbits && q < T) {
      fix_tail(q);
      wait_lgkm0();
    }
    raw_barrier();
    // (2) Y partial of tile q (waves w < NB2: N block w; two accumulators),
    // stored column major: column 32 w + l32, rows 8 j + 4 hl .. + 3
    {
      f32x16_t yp = f32x16_t{};
      if (q < T && w < NB2) {
        const uint8_t* xb = xs + (int)(q % FXB) * XTB;
        f32x16_t ya0 = f32x16_t{}, ya1 = f32x16_t{};
#pragma unroll
        for (int s = 0; s < 16; s += 2) {
          const uint4 a0 = *reinterpret_cast<const uint4*>(
              xb + l32 * 512 + (((2 * s + hl) ^ (l32 & 7)) * 16));
          const uint4 a1 = *reinterpret_cast<const uint4*>(
              xb + l32 * 512 + (((2 * s + 2 + hl) ^ (l32 & 7)) * 16));
          ya0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(a0), as_bf16x8(vf[s]), ya0, 0, 0,
                                                        0);
          ya1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(a1), as_bf16x8(vf[s + 1]), ya1,
                                                        0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) yp[i] = ya0[i] + ya1[i];
      }
      const bool real = q < T && w < NB2;
      float* dst = real ? ex_slot(q, m) + (int64_t)(32 * w + l32) * FR + 4 * hl : dummy + t * 16;
      const int step = real ? 8 : 4;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        *reinterpret_cast<float4*>(dst + j * step) =
            make_float4(yp[4 * j], yp[4 * j + 1], yp[4 * j + 2], yp[4 * j + 3]);
    }
    // (3) every member has posted iteration q-2: its partial of tile q-2 and
    // its bf16 slice of tile q-5 are in L2
    if (w == 0 && q >= 2 && !__all(seen >= want) &&
        !wait_members<C>(words, want, abort_word, spin_limit) && lane == 0)
      s_ctl[0] = 1;
    raw_barrier();
    if (s_ctl[0]) {
      set_status(status, PPCA_ERR_TIMEOUT);
      break;
    }
    // (4) loads of the reduction of tile q-2: this member's column block
    const bool red = q >= 2 && q - 2 < T;
    float4 rv[RIT][C];
#pragma unroll
    for (int it = 0; it < RIT; ++it) {
      const int item = t + 256 * it;
      const int kc = m * KPC + (item < ITEMS ? item / 8 : 0);
      const int rq = item % 8;
#pragma unroll
      for (int mm = 0; mm < C; ++mm) {
        const int64_t off = red ? ((ex_slot(q - 2, mm) - ex) + (int64_t)kc * FR + 4 * rq) * 4 : 0;
        rv[it][mm] = __builtin_bit_cast(
            float4, __builtin_amdgcn_raw_buffer_load_b128(exr, (int)off, 0, 16));
      }
    }
    // (5) bf16 Y tile q-5 -> LDS slot (q-5) & 1
    {
      const bool cp = q >= 5 && q - 5 < T;
      const uint8_t* src = reinterpret_cast<const uint8_t*>(cp ? yb_slot(q - 5) : ybg);
      uint8_t* dst = ys + (int)((q + 1) & 1) * YSB;
#pragma unroll
      for (int jj = 0; jj < YDPW; ++jj) {
        int off = ((jj * 4 + w) * 64 + lane) * 16;
        if (off >= YTB) off = 0;
        dma16_sc1(src + off, dst + (jj * 4 + w) * 1024);
      }
    }
    // (6) Z += X(q-6)^T Y(q-6)
    if (q >= 6 && q - 6 < T) {
      wait_vmcnt<W_Y>();
      raw_barrier();
      const uint8_t* xb = xs + (int)((q - 6) % FXB) * XTB;
      const uint8_t* yl = ys + (int)(q & 1) * YSB;
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        // A: columns 64 w + 2 l32 (+1) of rows 16 ks + 8 hl + e, e = 0..7
        uint32_t in[8];
        const int ch = 8 * w + (l32 >> 2);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int row = 16 * ks + 8 * hl + e;
          in[e] = *reinterpret_cast<const uint32_t*>(xb + row * 512 + ((ch ^ (row & 7)) * 16) +
                                                     (l32 & 3) * 4);
        }
        const uint4 a0 = make_uint4((in[0] & 0xFFFFu) | (in[1] << 16),
                                    (in[2] & 0xFFFFu) | (in[3] << 16),
                                    (in[4] & 0xFFFFu) | (in[5] << 16),
                                    (in[6] & 0xFFFFu) | (in[7] << 16));
        const uint4 a1 = make_uint4((in[0] >> 16) | (in[1] & 0xFFFF0000u),
                                    (in[2] >> 16) | (in[3] & 0xFFFF0000u),
                                    (in[4] >> 16) | (in[5] & 0xFFFF0000u),
                                    (in[6] >> 16) | (in[7] & 0xFFFF0000u));
#pragma unroll
        for (int nb = 0; nb < NB2; ++nb) {
          // B: rows 16 ks + 8 hl .. + 7 of column 32 nb + l32 (one 16-byte chunk)
          const uint4 bv = *reinterpret_cast<const uint4*>(
              yl + ((2 * ks + hl) * Kp + 32 * nb + l32) * 16);
          zacc[0][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(a0), as_bf16x8(bv),
                                                                zacc[0][nb], 0, 0, 0);
          zacc[1][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(a1), as_bf16x8(bv),
                                                                zacc[1][nb], 0, 0, 0);
        }
      }
    }
    // (7) reduction of tile q-2: sum in member order, rows past the pass are
    // zero, round to bf16, store this member's slice
    wait_vmcnt<W_R>();
#pragma unroll
    for (int it = 0; it < RIT; ++it) {
      const int item = t + 256 * it;
      const bool act = red && item < ITEMS;
      float4 sm = rv[it][0];
#pragma unroll
      for (int mm = 1; mm < C; ++mm) {
        sm.x += rv[it][mm].x;
        sm.y += rv[it][mm].y;
        sm.z += rv[it][mm].z;
        sm.w += rv[it][mm].w;
      }
      const int kc = m * KPC + (item < ITEMS ? item / 8 : 0);
      const int rq = item % 8;
      const int64_t i0 = red ? tile_row0(q - 2) + 4 * rq : 0;
      const float v0 = i0 < rows ? sm.x : 0.f, v1 = i0 + 1 < rows ? sm.y : 0.f;
      const float v2 = i0 + 2 < rows ? sm.z : 0.f, v3 = i0 + 3 < rows ? sm.w : 0.f;
      uint2 wv;
      wv.x = f32_to_bf16_bits(v0) | (f32_to_bf16_bits(v1) << 16);
      wv.y = f32_to_bf16_bits(v2) | (f32_to_bf16_bits(v3) << 16);
      uint2* dst = act ? reinterpret_cast<uint2*>(yb_slot(q - 2) +
                                                  ((rq >> 1) * Kp + kc) * 8 + (rq & 1) * 4)
                       : reinterpret_cast<uint2*>(dummy + 4096 + t * 4 + it * 2);
      *dst = wv;
    }
    // (8) post iteration q: the partial of tile q (stored before the reduction
    // loads, which have returned) and the slice of tile q-3 (stored in the
    // previous iteration, before those loads) are complete in every wave.  The
    // X buffer of tile q-6 is free: tile q+2 goes there.
    raw_barrier();
    if (t == 0) __hip_atomic_store(words + m, (int)(q + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    issue_x(q + 2);
  }
  wait_vmcnt<0>();

  // ---- Z partial of this (slice, cluster): part[m][cl][Kp][256]; element i of
  // zacc[v][nb] is slice column 64 w + 2 (8 (i / 4) + 4 hl + i % 4) + v, Y column 32 nb + l32
  float* zp = part + ((int64_t)m * NCL + cl) * Kp * FSW;
#pragma unroll
  for (int v = 0; v < 2; ++v)
#pragma unroll
    for (int nb = 0; nb < NB2; ++nb)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int mu = 8 * (i / 4) + 4 * hl + (i % 4);
        zp[(int64_t)(32 * nb + l32) * FSW + 64 * w + 2 * mu + v] = zacc[v][nb][i];
      }
}

template <typename F>
hipError_t dispatch_fused(int Kp, int C, F&& f) {
  auto byc = [&](auto nb2) -> hipError_t {
    switch (C) {
      case 1: return f(nb2, std::integral_constant<int, 1>{});
      case 2: return f(nb2, std::integral_constant<int, 2>{});
      case 4: return f(nb2, std::integral_constant<int, 4>{});
      case 8: return f(nb2, std::integral_constant<int, 8>{});
      case 16: return f(nb2, std::integral_constant<int, 16>{});
      case 32: return f(nb2, std::integral_constant<int, 32>{});
      default: return hipErrorInvalidValue;
    }
  };
  switch (Kp) {
    case 32: return byc(std::integral_constant<int, 1>{});
    case 64: return byc(std::integral_constant<int, 2>{});
    case 96: return byc(std::integral_constant<int, 3>{});
    case 128: return byc(std::integral_constant<int, 4>{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int fused_cluster(int64_t d) {
  int c = 1;
  while ((int64_t)c * FSW < d) c *= 2;
  return c;
}

FusedSizes fused_sizes(int64_t d, int Kp) {
  FusedSizes z{};
  const int C = fused_cluster(d);
  const int ncl = 256 / C;
  z.cluster = C;
  z.ex_bytes = (size_t)ncl * FSLOT * C * Kp * FR * 4;
  z.yb_bytes = (size_t)ncl * FSLOT * 4 * Kp * 16;
  z.flag_bytes = ((size_t)ncl + 8 + 1) * FFLAG * 4;
  z.dummy_bytes = (size_t)8192 * 4;
  z.part_bytes = (size_t)C * ncl * Kp * FSW * 4;
  z.nsplit = ncl;
  return z;
}

bool fused_eligible(int32_t dtype, int64_t d, int Kp) {
  return dtype == PPCA_BF16 && Kp % 32 == 0 && Kp <= 128 && d <= (int64_t)32 * FSW;
}

hipError_t launch_fused_pass(const PassDesc& p, const void* vop, int64_t dp, int Kp,
                             const FusedBufs& fb, int* status, int spin_limit, hipStream_t s) {
  const int C = fused_cluster(p.d);
  hipError_t e = launch_zero(fb.flags, fused_sizes(p.d, Kp).flag_bytes, s);
  if (e != hipSuccess) return e;
  return dispatch_fused(Kp, C, [&](auto nb2, auto cc) {
    constexpr int NB2 = decltype(nb2)::value, CC = decltype(cc)::value;
    const uint8_t* x = (const uint8_t*)p.x;
    int64_t n = p.n, d = p.d, ld = p.ld, r0 = p.r0, rows = p.nrows;
    const uint8_t* v = (const uint8_t*)vop;
    int64_t dpp = dp;
    float* ex = fb.ex;
    uint16_t* yb = fb.yb;
    int* fl = fb.flags;
    float* dm = fb.dummy;
    float* pt = fb.part;
    int* st = status;
    int sl = spin_limit;
    void* args[] = {&x, &n, &d, &ld, &r0, &rows, &v, &dpp, &ex, &yb, &fl, &dm, &pt, &st, &sl};
    return hipLaunchCooperativeKernel((const void*)k_xxv<NB2, CC>, dim3(256), dim3(256), args, 0,
                                      s);
  });
}

}  // namespace ppca
