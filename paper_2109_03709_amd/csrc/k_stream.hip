// Streaming kernels of one pass over X (block power step, minibatch step and
// pPCA projection, Alg. 1 steps 2-3 and Sec. 2.1):
//
//   k_xvd     : Y = X V' and the partial Grams G_w = Y^T Y of workgroup w
//               (bf16 / f32 data; persistent over row tiles, full d per tile,
//               LDS-DMA stages)
//   k_xv      : the same for fp8 data (register-staged pipeline; fp8 codes
//               are widened to bf16 exactly when read from LDS)
//   k_xvy     : Y = X V' of the power pass for bf16 data (one DMA pipeline
//               over all tiles of a workgroup, Y stored from the accumulators)
//   k_ysum    : short passes (few 64-row tiles) split their columns over
//               several workgroups of k_xvd / k_xv in partial mode; this sums
//               the float32 Y partials, writes Y and the G partials
//   k_xtyd    : Z = X^T Y over (256-column tile, row split) pairs (LDS-DMA)
//   reduce_zg : fixed-order float64 sum of the partials -> Z (f32), G (f64)
//
// The projection pass only needs G, so it runs the Y = X V' kernel alone
// (one read of X, no Y written).  The power pass of bf16 data with Kp a
// multiple of 32 over 256-row tiles (k_xvy) runs on v_mfma_f32_32x32x16_bf16
// (with one wave per SIMD it sustains about 2.5 times the rate of the 16x16
// shapes); the other products of bf16 and fp8 data on
// v_mfma_f32_16x16x32_bf16 (for X^T Y, whose A operand is a transpose read
// from LDS, the 32x32 shape measured slower), float32 data on
// v_mfma_f32_16x16x4_f32.
// Accumulation inside a workgroup is float32; partials are summed in float64
// in a fixed order, so results are bitwise reproducible run to run.
//
// Layouts
//   X     row-major [n][ld] (element type per dtype); pass row i is data row
//         (r0 + i) mod n.
//   V'^T  operand [Kp][dp] (bf16 or f32), zero padded in both directions
//         (dp a multiple of 64).
//   Y     "blocked" staging buffer so that the X^T Y kernel reads 8 (bf16) or
//         4 (f32) consecutive rows of one Y column as one 16-byte chunk:
//         bf16: yb[row/8][Kp][8], f32: yb[row/4][Kp][4].
//   part  [tile][split][Kp][256] float32: column c of tile t is column
//         t*256 + c of X.
//   gpart [workgroup of the Y = X V' kernel, or of k_ysum][Kp][Kp] float32.
//   ypart [split][rows rounded to 64][Kp] float32 (short passes only).
#include "lds_dma.h"

namespace ppca {

namespace {

using namespace dma;

constexpr int DT_F32 = 0, DT_BF16 = 1, DT_FP8 = 2;

// widen 4 fp8 codes (one dword) to 4 bf16 (two dwords)
__device__ inline uint2 fp8x4_to_bf16x4(uint32_t w) {
  uint2 r;
  r.x = e4m3_to_bf16_bits(w & 0xFF) | (e4m3_to_bf16_bits((w >> 8) & 0xFF) << 16);
  r.y = e4m3_to_bf16_bits((w >> 16) & 0xFF) | (e4m3_to_bf16_bits(w >> 24) << 16);
  return r;
}

// Mask of the elements of a 16-byte chunk (EB bytes per element) whose
// column index col + e is below d: whole words are kept or cleared, a word
// holding a valid and an invalid element keeps its low half.
template <int EB>
__device__ inline uint4 chunk_mask(int64_t col, int64_t d) {
  constexpr int NE = 16 / EB;
  int64_t nv = d - col;
  nv = nv < 0 ? 0 : (nv > NE ? NE : nv);
  const int v = (int)nv * EB;              // valid bytes in the chunk
  uint32_t w[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int b = v - 4 * i;               // valid bytes in word i
    w[i] = b >= 4 ? 0xFFFFFFFFu : (b <= 0 ? 0u : (0xFFFFFFFFu >> (8 * (4 - b))));
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// Slot of chunk c of a 128-byte LDS row r is c ^ swz(r).  A 128-bit LDS read
// serves 16 lanes per pass from the 64 banks (16 units of 16 bytes); unit of
// (r, slot) = 8 (r & 1) + slot.  The fragment reads take one chunk of 16
// consecutive rows r0 .. r0 + 15 (r0 a multiple of 16), and (r >> 1) & 7
// gives those rows 16 distinct units (r & 7 gave rows r and r + 8 the same
// unit: a two-way conflict on every read).
__device__ inline int swz(int r) { return (r >> 1) & 7; }

__device__ inline uint4 and4(uint4 a, uint4 m) {
  return make_uint4(a.x & m.x, a.y & m.y, a.z & m.z, a.w & m.w);
}

// LDS swizzles of the k_xv stages (LDS: 128 bytes per cycle over 32 banks;
// a 16-byte read serves 8 lanes per pass, an 8-byte read 16 lanes).
// 64-byte rows (bf16 X, V', f32 X): chunk c of row r sits at c ^ sw64(r), so
// that the 8 consecutive rows read by one pass (and the 16 of a 256-byte
// pass) land on distinct 16-byte bank groups.
__device__ inline int sw64(int r) { return ((r >> 1) ^ (r >> 3)) & 3; }
// 32-byte rows (fp8 X): 8-byte piece p of row r sits at p ^ sw32(r), so that
// the 16 rows read by one 8-byte pass land on distinct 8-byte bank groups.
__device__ inline int sw32(int r) { return (r >> 2) & 3; }

// ---------------------------------------------------------------------------
// Y = X V' and G = Y^T Y.  Persistent: workgroup w takes the row tiles
// w, w + gridDim.x, ... (WGR = 4 waves x MW x 16 rows each).  Per tile, the
// k-loop (32 columns per step, 16 for f32) runs a software pipeline: the X and
// V' tiles of a step are loaded into registers PSX-1 steps ahead (PSX register
// stages), written to one of two LDS buffers one step ahead and consumed by
// the MFMAs; one barrier per step.  After the k-loop the tile of Y goes to
// LDS (over the pipeline buffers, blocked layout below), is copied to global
// memory when the pass needs it (WANT_Y) and feeds G += Y^T Y.  The G
// accumulators of a lane live in LDS slots private to that lane between
// tiles (they are only needed in the tile epilogue), which leaves the
// register file to the Y accumulators and the in-flight stages; the G
// partial of the workgroup is written once at the end.
// ---------------------------------------------------------------------------
template <int... I, typename F>
__device__ __attribute__((always_inline)) inline void unroll_seq(std::integer_sequence<int, I...>, F&& f) {
  (f(std::integral_constant<int, I>{}), ...);
}

// The streamed pointers are deliberately not __restrict__: loads through
// restrict-qualified read-only kernel arguments may be moved down to their
// use, which would collapse the pipeline.
template <int NB, int DT, int MW, int PSX, bool WANT_Y, bool WANT_G, bool PART = false>
__global__ __launch_bounds__(256, 1) void k_xv(const uint8_t* x_, int64_t n, int64_t d_, int64_t ld,
                                               int64_t rstart, int64_t rows, const uint8_t* vop_,
                                               int64_t dp, uint8_t* yb, float* gpart,
                                               int accumulate, float* ypart, int64_t yrows) {
  static_assert(!PART || (!WANT_Y && !WANT_G), "partial mode writes only float32 Y partials");
  constexpr int Kp = NB * 16;
  constexpr int NBG = (NB + 3) / 4;                               // G column blocks per wave
  constexpr int EB = DT == DT_F32 ? 4 : DT == DT_BF16 ? 2 : 1;   // bytes per X element
  constexpr int OB = DT == DT_F32 ? 4 : 2;                        // bytes per operand element
  constexpr int YB = OB;                                          // bytes per Y element
  constexpr int YR = 16 / YB;                                     // rows per Y chunk (8 or 4)
  constexpr int KS = DT == DT_F32 ? 16 : 32;                      // columns per k-step
  constexpr int WGR = 4 * MW * 16;                                // rows per tile
  constexpr int XCPR = KS * EB / 16;                              // 16-B chunks per X row (4 or 2)
  constexpr int XSTB = WGR * XCPR * 16;                           // X bytes per stage
  constexpr int XCHT = XSTB / 16;                                 // X chunks per stage
  constexpr int XCH = (XCHT + 255) / 256;                         // X chunks per thread
  constexpr int VSTB = Kp * 64;                                   // V' bytes per stage (4 chunks/row)
  constexpr int VCH = (Kp * 4 + 255) / 256;                       // V' chunks per thread
  constexpr int YTB = WGR * Kp * YB;                              // Y tile bytes
  constexpr int YTCHT = YTB / 16;                                 // Y tile chunks
  constexpr int PIPEB = 2 * (XSTB + VSTB);
  constexpr int REGA = PIPEB > YTB ? PIPEB : YTB;                 // pipeline buffers / Y tile
  constexpr int GSLOT = WANT_G ? NB * NBG * 4 * 64 * 16 : 16;    // G accumulator slots
  static_assert(PSX % 2 == 0, "the LDS buffer of a step is its parity");
  __shared__ __attribute__((aligned(16))) uint8_t lds[REGA + GSLOT];
  uint8_t* const ylds = lds;
  f32x4_t* const gslot = reinterpret_cast<f32x4_t*>(lds + REGA);

  // partial mode (split of the columns, blockIdx.y = split), as in k_xvd
  const uint8_t* x = x_;
  const uint8_t* vop = vop_;
  int64_t d = d_;
  if constexpr (PART) {
    const int nk_all = (int)((d_ + KS - 1) / KS);
    const int kper = (nk_all + (int)gridDim.y - 1) / (int)gridDim.y;
    const int64_t c0 = (int64_t)blockIdx.y * kper * KS;
    if (c0 >= d_) return;                    // uniform; excluded by the split count
    x += c0 * EB;
    vop += c0 * OB;
    d = d_ - c0 < (int64_t)kper * KS ? d_ - c0 : (int64_t)kper * KS;
  }
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int a = lane & 15, g = lane >> 4;
  const uint32_t keep = dp > 0 ? 0xFFFFFFFFu : 0u;   // all ones, opaque to the compiler
  const int64_t ntile = (rows + WGR - 1) / WGR;

  // lane-private G slot of block (mb, q): ((mb * NBG + q) * 4 + wave) * 64 + lane
  auto gs = [&](int mb, int q) __attribute__((always_inline)) -> f32x4_t& { return gslot[((mb * NBG + q) * 4 + wave) * 64 + lane]; };
  if (WANT_G) {
#pragma unroll
    for (int mb = 0; mb < NB; ++mb)
#pragma unroll
      for (int q = 0; q < NBG; ++q) gs(mb, q) = f32x4_t{0.f, 0.f, 0.f, 0.f};
  }

  // X chunk s of a stage = (row s / XCPR, chunk s % XCPR), swizzled in LDS;
  // threads past the last chunk repeat an earlier one (identical writes)
  // (fp8: the two 8-byte halves of a chunk go to xdst and xdst2)
  int xrow[XCH], xdst[XCH], xdst2[XCH], xcol[XCH];
#pragma unroll
  for (int j = 0; j < XCH; ++j) {
    const int s = (t + 256 * j) % XCHT, r = s / XCPR, c = s % XCPR;
    xrow[j] = r;
    xcol[j] = c * (16 / EB);
    if (XCPR == 4) {
      xdst[j] = (r * 4 + (c ^ sw64(r))) * 16;
      xdst2[j] = 0;
    } else {
      xdst[j] = r * 32 + ((2 * c) ^ sw32(r)) * 8;
      xdst2[j] = r * 32 + ((2 * c + 1) ^ sw32(r)) * 8;
    }
  }
  // V' chunks: threads past the last chunk repeat an earlier one
  const uint8_t* vsrc[VCH];
  int vdst[VCH];
#pragma unroll
  for (int j = 0; j < VCH; ++j) {
    const int s = (t + 256 * j) % (Kp * 4), r = s >> 2, c = s & 3;
    vsrc[j] = vop + ((int64_t)r * dp) * OB + c * 16;
    vdst[j] = (r * 4 + (c ^ sw64(r))) * 16;
  }

  // Y accumulators: zeroed once here and cleared at the end of each tile
  f32x4_t acc[MW][NB];
#pragma unroll
  for (int mb = 0; mb < MW; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  for (int64_t tl = blockIdx.x; tl < ntile; tl += gridDim.x) {
    const int64_t row0 = tl * WGR;
    // per-tile row sources: rows past the pass read a valid row, masked at the LDS write
    const uint8_t* xsrc[XCH];
    uint32_t xrowm[XCH];
#pragma unroll
    for (int j = 0; j < XCH; ++j) {
      const int64_t li = row0 + xrow[j];
      const bool ok = li < rows;
      xrowm[j] = ok ? 0xFFFFFFFFu : 0u;
      xsrc[j] = x + ((rstart + (ok ? li : 0)) % n) * ld * EB;
    }

    uint4 xr[PSX][XCH], vr[PSX][VCH];
    auto gload = [&](int64_t k0, uint4 (&xo)[XCH], uint4 (&vo)[VCH]) __attribute__((always_inline)) {
#pragma unroll
      for (int j = 0; j < XCH; ++j) {
        const int64_t col = k0 + xcol[j];
        const int64_t ce = col < d ? col : 0;
        xo[j] = *reinterpret_cast<const uint4*>(xsrc[j] + ce * EB);
      }
#pragma unroll
      for (int j = 0; j < VCH; ++j) vo[j] = *reinterpret_cast<const uint4*>(vsrc[j] + k0 * OB);
    };
    // mask (rows past the pass, columns past d) and write one stage to LDS;
    // the AND on V' also keeps the compiler from fusing load and store into a
    // memcpy placed here (which would move the load down to this point)
    auto lwrite = [&](int buf, int64_t k0, const uint4 (&xi)[XCH], const uint4 (&vi)[VCH]) __attribute__((always_inline)) {
      uint8_t* xs = lds + buf * (XSTB + VSTB);
      uint8_t* vs = xs + XSTB;
#pragma unroll
      for (int j = 0; j < XCH; ++j) {
        uint4 m = chunk_mask<EB>(k0 + xcol[j], d);
        m = make_uint4(m.x & xrowm[j], m.y & xrowm[j], m.z & xrowm[j], m.w & xrowm[j]);
        const uint4 v = and4(xi[j], m);
        if (XCPR == 4) {
          *reinterpret_cast<uint4*>(xs + xdst[j]) = v;
        } else {
          *reinterpret_cast<uint2*>(xs + xdst[j]) = make_uint2(v.x, v.y);
          *reinterpret_cast<uint2*>(xs + xdst2[j]) = make_uint2(v.z, v.w);
        }
      }
#pragma unroll
      for (int j = 0; j < VCH; ++j)
        *reinterpret_cast<uint4*>(vs + vdst[j]) = and4(vi[j], make_uint4(keep, keep, keep, keep));
    };

    auto compute = [&](int buf) __attribute__((always_inline)) {
      const uint8_t* xs = lds + buf * (XSTB + VSTB);
      const uint8_t* vs = xs + XSTB;
      if (DT == DT_F32) {
        float4 af[MW], bf[NB];
#pragma unroll
        for (int mb = 0; mb < MW; ++mb) {
          const int r = wave * MW * 16 + mb * 16 + a;
          af[mb] = *reinterpret_cast<const float4*>(xs + (r * 4 + (g ^ sw64(r))) * 16);
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const int r = nb * 16 + a;
          bf[nb] = *reinterpret_cast<const float4*>(vs + (r * 4 + (g ^ sw64(r))) * 16);
        }
#pragma unroll
        for (int mb = 0; mb < MW; ++mb)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mb].x, bf[nb].x, acc[mb][nb], 0, 0, 0);
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mb].y, bf[nb].y, acc[mb][nb], 0, 0, 0);
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mb].z, bf[nb].z, acc[mb][nb], 0, 0, 0);
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mb].w, bf[nb].w, acc[mb][nb], 0, 0, 0);
          }
      } else {
        uint4 af[MW], bf[NB];
#pragma unroll
        for (int mb = 0; mb < MW; ++mb) {
          const int r = wave * MW * 16 + mb * 16 + a;
          if (DT == DT_FP8) {
            const uint2 w = *reinterpret_cast<const uint2*>(xs + r * 32 + (g ^ sw32(r)) * 8);
            const uint2 lo = fp8x4_to_bf16x4(w.x), hi = fp8x4_to_bf16x4(w.y);
            af[mb] = make_uint4(lo.x, lo.y, hi.x, hi.y);
          } else {
            af[mb] = *reinterpret_cast<const uint4*>(xs + (r * 4 + (g ^ sw64(r))) * 16);
          }
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const int r = nb * 16 + a;
          bf[nb] = *reinterpret_cast<const uint4*>(vs + (r * 4 + (g ^ sw64(r))) * 16);
        }
#pragma unroll
        for (int mb = 0; mb < MW; ++mb)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(af[mb]), as_bf16x8(bf[nb]),
                                                                  acc[mb][nb], 0, 0, 0);
      }
    };

    // Straight-line loop body (a branch between a stage's loads and its LDS
    // write lets the compiler sink the loads to their use).  Steps past the
    // last one load a clamped, valid stage and write it with an all-zero
    // column mask, so their MFMAs add exactly zero.
    const int nk = (int)((d + KS - 1) / KS);
    const int64_t klast = (int64_t)(nk - 1) * KS;
#pragma unroll
    for (int i = 0; i < PSX - 1; ++i) gload(min((int64_t)i * KS, klast), xr[i], vr[i]);
    lwrite(0, 0, xr[0], vr[0]);
    __syncthreads();
    for (int k = 0; k < nk; k += PSX) {
      unroll_seq(std::make_integer_sequence<int, PSX>{}, [&](auto I) __attribute__((always_inline)) {
        constexpr int i = decltype(I)::value;
        const int kk = k + i;
        gload(min((int64_t)(kk + PSX - 1) * KS, klast), xr[(i + PSX - 1) % PSX], vr[(i + PSX - 1) % PSX]);
        __builtin_amdgcn_sched_barrier(0);
        compute(i & 1);
        __builtin_amdgcn_sched_barrier(0);
        lwrite((i + 1) & 1, (int64_t)(kk + 1) * KS, xr[(i + 1) % PSX], vr[(i + 1) % PSX]);
        __syncthreads();
      });
    }

    if constexpr (PART) {
      // float32 partial of this split: ypart[split][row0 + lr][c]
      float* yp = ypart + ((int64_t)blockIdx.y * yrows + row0) * Kp;
#pragma unroll
      for (int mb = 0; mb < MW; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int u = 0; u < 4; ++u)
            yp[(int64_t)(wave * MW * 16 + mb * 16 + 4 * g + u) * Kp + nb * 16 + a] = acc[mb][nb][u];
    } else {
    // ---- Y tile -> LDS (over the pipeline buffers: the last barrier of the
    // k-loop ended every read of them), layout [row/YR][Kp][YR].
    // D[i][j]: lane (j = a, g) holds rows 4g..4g+3 of each 16-row block.
#pragma unroll
    for (int mb = 0; mb < MW; ++mb) {
      const int lr = wave * MW * 16 + mb * 16 + 4 * g;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        if (DT == DT_F32) {
          *reinterpret_cast<float4*>(ylds + ((lr >> 2) * Kp + nb * 16 + a) * 16) =
              make_float4(acc[mb][nb][0], acc[mb][nb][1], acc[mb][nb][2], acc[mb][nb][3]);
        } else {
          uint2 w;
          w.x = f32_to_bf16_bits(acc[mb][nb][0]) | (f32_to_bf16_bits(acc[mb][nb][1]) << 16);
          w.y = f32_to_bf16_bits(acc[mb][nb][2]) | (f32_to_bf16_bits(acc[mb][nb][3]) << 16);
          *reinterpret_cast<uint2*>(ylds + ((lr >> 3) * Kp + nb * 16 + a) * 16 + (lr & 7) * 2) = w;
        }
      }
    }
    __syncthreads();
    if (WANT_Y) {
      // coalesced copy of the tile to the global staging buffer (same layout)
      uint8_t* ydst = yb + row0 * Kp * YB;
      for (int s = t; s < YTCHT; s += 256)
        *reinterpret_cast<uint4*>(ydst + s * 16) = *reinterpret_cast<const uint4*>(ylds + s * 16);
    }
    // G += Y^T Y over the tile's rows; wave w takes the column blocks nb = w (mod 4)
    // (rows past the pass are zero in Y because their X rows were masked)
    if constexpr (WANT_G) {
    constexpr int GS = DT == DT_F32 ? 4 : 8;                       // rows per lane group
    f32x4_t accg[NB][NBG];
#pragma unroll
    for (int mb = 0; mb < NB; ++mb)
#pragma unroll
      for (int q = 0; q < NBG; ++q) accg[mb][q] = gs(mb, q);
    // B fragments of the wave's blocks nb = wave + 4q are read by address (a
    // register array indexed by the wave number would live in scratch);
    // blocks past NB read block 0 and their products are never stored
#pragma unroll
    for (int r0 = 0; r0 < WGR; r0 += 4 * GS) {
      const int rg = r0 / YR + g;                                  // chunk row of this lane group
      const uint8_t* yrow = ylds + (rg * Kp + a) * 16;
      if (DT == DT_F32) {
        float4 ya[NB], yw[NBG];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) ya[nb] = *reinterpret_cast<const float4*>(yrow + nb * 256);
#pragma unroll
        for (int q = 0; q < NBG; ++q) {
          const int nb = wave + 4 * q;
          yw[q] = *reinterpret_cast<const float4*>(yrow + (nb < NB ? nb : 0) * 256);
        }
#pragma unroll
        for (int mb = 0; mb < NB; ++mb)
#pragma unroll
          for (int q = 0; q < NBG; ++q) {
            accg[mb][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ya[mb].x, yw[q].x, accg[mb][q], 0, 0, 0);
            accg[mb][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ya[mb].y, yw[q].y, accg[mb][q], 0, 0, 0);
            accg[mb][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ya[mb].z, yw[q].z, accg[mb][q], 0, 0, 0);
            accg[mb][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ya[mb].w, yw[q].w, accg[mb][q], 0, 0, 0);
          }
      } else {
        uint4 ya[NB], yw[NBG];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) ya[nb] = *reinterpret_cast<const uint4*>(yrow + nb * 256);
#pragma unroll
        for (int q = 0; q < NBG; ++q) {
          const int nb = wave + 4 * q;
          yw[q] = *reinterpret_cast<const uint4*>(yrow + (nb < NB ? nb : 0) * 256);
        }
#pragma unroll
        for (int mb = 0; mb < NB; ++mb)
#pragma unroll
          for (int q = 0; q < NBG; ++q)
            accg[mb][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ya[mb]), as_bf16x8(yw[q]),
                                                                  accg[mb][q], 0, 0, 0);
      }
    }
#pragma unroll
    for (int mb = 0; mb < NB; ++mb)
#pragma unroll
      for (int q = 0; q < NBG; ++q) gs(mb, q) = accg[mb][q];
    }
    }   // !PART
    // clear the accumulators for the next tile with a zero the compiler cannot
    // see through (a literal zero at the top of the tile makes the register
    // allocator rotate the accumulators through extra registers in the k-loop)
    const float zero = __uint_as_float(~keep);
#pragma unroll
    for (int mb = 0; mb < MW; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4_t{zero, zero, zero, zero};
    __syncthreads();   // the next tile's pipeline overwrites the Y tile
  }
  if (!WANT_G) return;

  // G partial of this workgroup: block (mb, nb), lane (j = a, g) holds rows
  // 16mb + 4g + u, column 16nb + a
  float* gbase = gpart + (int64_t)blockIdx.x * Kp * Kp;
#pragma unroll
  for (int mb = 0; mb < NB; ++mb)
#pragma unroll
    for (int q = 0; q < NBG; ++q) {
      const int nb = wave + 4 * q;
      if (nb >= NB) continue;
      const f32x4_t v = gs(mb, q);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        float* p = gbase + (int64_t)(mb * 16 + 4 * g + u) * Kp + nb * 16 + a;
        if (accumulate) *p += v[u];   // chunked passes only
        else *p = v[u];
      }
    }
}

// ---------------------------------------------------------------------------
// Y = X V' and G = Y^T Y with LDS-DMA stages (bf16 and f32 data).
//
// Same work split as k_xv (persistent workgroups over tiles of WGR rows, full
// d per tile), but the k-step covers 128 bytes of every row (64 bf16 / 32 f32
// columns: whole cache lines) and its X and V' tiles go straight from global
// memory to LDS with global_load_lds (no register staging), into three LDS
// stages kept as separate arrays:
//   step kk:  wait for this wave's DMA of step kk (step kk+1 stays in flight)
//             -> barrier -> DMA of step kk+2 into the stage freed by step kk-1
//             -> MFMAs on stage kk.
// A DMA writes 64 lanes x 16 bytes to consecutive LDS slots, so the XOR
// swizzle of a 128-byte row (chunk c at slot c ^ swz(row)) is produced by
// choosing which global chunk each lane loads.
// Every wave issues the same number of DMAs per step (steps past the last one
// and the V' blocks of a small K repeat valid loads), so a fixed vmcnt wait
// always means "the stage I need has landed".
// Rows past the pass load a valid row; their Y rows are zeroed in the
// epilogue.  A last step that ends inside a 16-byte chunk has the chunk's
// columns past d cleared in LDS by the lane that loaded it.
// ---------------------------------------------------------------------------
template <int NB, int DT, int MW, bool WANT_Y, bool WANT_G, bool PART = false, bool SPLIT = false>
__global__ __launch_bounds__(256, 1) void k_xvd(const uint8_t* x_, int64_t n, int64_t d_, int64_t ld,
                                                int64_t rstart, int64_t rows, const uint8_t* vop_,
                                                int64_t dp, uint8_t* yb, float* gpart,
                                                int accumulate, float* ypart, int64_t yrows) {
  static_assert(DT == DT_F32 || DT == DT_BF16, "bf16 or f32 data");
  static_assert(!PART || (!WANT_Y && !WANT_G), "partial mode writes only float32 Y partials");
  // SPLIT: the two-term operand of the projection (hi at vop, lo Kp dp later),
  // two products per output into one float32 accumulator (partial mode only)
  static_assert(!SPLIT || (PART && DT == DT_BF16), "two-term operand: bf16 partial mode");
  constexpr int NV = SPLIT ? 2 : 1;                    // operand terms
  constexpr int Kp = NB * 16;
  constexpr int NBG = (NB + 3) / 4;                    // G column blocks per wave
  constexpr int EB = DT == DT_F32 ? 4 : 2;             // bytes per X / V' / Y element
  constexpr int KS = 128 / EB;                         // columns per k-step
  constexpr int WGR = 64 * MW;                         // rows per tile
  constexpr int XSB = WGR * 128, VSB = Kp * 128;       // stage bytes of X and V'
  constexpr int STB = XSB + NV * VSB;
  constexpr int XI = WGR / 32;                         // X DMAs per wave per step
  constexpr int VBLK = Kp / 8;                         // 1 KB blocks of a V' stage
  constexpr int VI = (VBLK + 3) / 4;                   // V' DMAs per wave per step
  constexpr int DPS = XI + NV * VI;                    // DMAs per wave per step
  constexpr int YR = 16 / EB;                          // rows per Y chunk (8 / 4)
  constexpr int YTB = WGR * Kp * EB;                   // Y tile bytes
  constexpr int YHB = YTB / 2;                         // half tile (rows [0, WGR/2) in st0)
  static_assert(PART || YHB <= STB, "a Y half tile fits a stage");   // partials skip LDS
  static_assert(2 * DPS < 64, "vmcnt range");
  __shared__ __attribute__((aligned(16))) uint8_t st0[STB];
  __shared__ __attribute__((aligned(16))) uint8_t st1[STB];
  __shared__ __attribute__((aligned(16))) uint8_t st2[STB];

  // partial mode (split of the columns): the split's k-steps [kper y,
  // kper (y + 1)) as a matrix of its own; the host picks the split count so
  // that every split has at least one k-step.  Its grid is (split, tile):
  // with a split count that is a multiple of 8, the workgroups of one split
  // (which all stream the same slice of V') share an XCD and its L2
  const int tb = PART ? (int)blockIdx.y : (int)blockIdx.x;   // tile workgroup
  const int tg = PART ? (int)gridDim.y : (int)gridDim.x;
  const int sb = PART ? (int)blockIdx.x : (int)blockIdx.y;   // split
  const int sg = PART ? (int)gridDim.x : (int)gridDim.y;
  const uint8_t* x = x_;
  const uint8_t* vop = vop_;
  int64_t d = d_;
  if constexpr (PART) {
    const int nk_all = (int)((d_ + KS - 1) / KS);
    const int kper = (nk_all + sg - 1) / sg;
    const int64_t c0 = (int64_t)sb * kper * KS;
    if (c0 >= d_) return;                    // uniform; excluded by the split count
    x += c0 * EB;
    vop += c0 * EB;
    d = d_ - c0 < (int64_t)kper * KS ? d_ - c0 : (int64_t)kper * KS;
  }
  const int t = threadIdx.x, lane = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int a = lane & 15, g = lane >> 4;
  const int64_t ntile = (rows + WGR - 1) / WGR;
  const int nk = (int)((d + KS - 1) / KS);
  const int64_t klast = (int64_t)(nk - 1) * KS;
  // a last k-step ending inside a 16-byte chunk needs its tail cleared
  const int64_t dtail = d % (16 / EB);
  const uint32_t keep = dp > 0 ? 0xFFFFFFFFu : 0u;     // all ones, opaque to the compiler

  // DMA sources.  X block j of wave w covers tile rows 8 (w XI + j) .. +7; lane
  // -> row 8 (w XI + j) + lane / 8, LDS slot lane % 8 holding chunk
  // (lane % 8) ^ swz(row).
  const int p8 = lane & 7;
  int xr[XI], xc[XI];
#pragma unroll
  for (int j = 0; j < XI; ++j) {
    const int r = 8 * (w * XI + j) + (lane >> 3);
    xr[j] = r;
    xc[j] = (p8 ^ swz(r)) * (16 / EB);                // first column of the chunk in the step
  }
  // data row of each X block row, advanced by (gridDim.x * WGR) mod n per
  // tile (any valid row serves the rows past the pass: they are zeroed later)
  const int64_t tstep = ((int64_t)tg * WGR) % n;
  int64_t xrow[XI];
#pragma unroll
  for (int j = 0; j < XI; ++j) xrow[j] = (rstart + (int64_t)tb * WGR + xr[j]) % n;
  const uint8_t* vsrc[VI];
  int vblk[VI];
#pragma unroll
  for (int j = 0; j < VI; ++j) {
    const int blk = (w * VI + j) % VBLK;
    const int r = 8 * blk + (lane >> 3);
    vblk[j] = blk;
    vsrc[j] = vop + (int64_t)r * dp * EB + (p8 ^ swz(r)) * 16;
  }

  f32x4_t acc[MW][NB];
#pragma unroll
  for (int mb = 0; mb < MW; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  f32x4_t accg[NB][NBG];
#pragma unroll
  for (int mb = 0; mb < NB; ++mb)
#pragma unroll
    for (int q = 0; q < NBG; ++q) accg[mb][q] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  for (int64_t tl = tb; tl < ntile; tl += tg) {
    const int64_t row0 = tl * WGR;
    const uint8_t* xsrc[XI];
#pragma unroll
    for (int j = 0; j < XI; ++j) {
      xsrc[j] = x + xrow[j] * ld * EB;
      const int64_t nr = xrow[j] + tstep;
      xrow[j] = nr >= n ? nr - n : nr;
    }
    auto stage = [&](int b) __attribute__((always_inline)) -> uint8_t* {
      return b == 0 ? st0 : (b == 1 ? st1 : st2);
    };
    // DMA of step kk (clamped to the last step) into stage b
    auto issue = [&](int kk, int b) __attribute__((always_inline)) {
      uint8_t* sb = stage(b);
      const int64_t k0 = kk < nk ? (int64_t)kk * KS : klast;
#pragma unroll
      for (int j = 0; j < XI; ++j) {
        const int64_t col = k0 + xc[j];
        dma16(xsrc[j] + (col < d ? col : 0) * EB, sb + (w * XI + j) * 1024);
      }
#pragma unroll
      for (int j = 0; j < VI; ++j) dma16(vsrc[j] + k0 * EB, sb + XSB + vblk[j] * 1024);
      if constexpr (SPLIT) {
        const int64_t lo_off = (int64_t)Kp * dp * EB;
#pragma unroll
        for (int j = 0; j < VI; ++j)
          dma16(vsrc[j] + lo_off + k0 * EB, sb + XSB + VSB + vblk[j] * 1024);
      }
    };
    // clear the columns past d of the chunks this lane loaded in the last step
    auto fix_tail = [&](int b) __attribute__((always_inline)) {
      uint8_t* sb = stage(b);
#pragma unroll
      for (int j = 0; j < XI; ++j) {
        uint4* slot = reinterpret_cast<uint4*>(sb + (w * XI + j) * 1024 + lane * 16);
        *slot = and4(*slot, chunk_mask<EB>(klast + xc[j], d));
      }
    };
    auto compute = [&](int b) __attribute__((always_inline)) {
      const uint8_t* xs = stage(b);
      const uint8_t* vs = xs + XSB;
      if (DT == DT_F32) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          float4 af[MW], bf[NB];
          const int c = 4 * q + g;
#pragma unroll
          for (int mb = 0; mb < MW; ++mb) {
            const int r = w * MW * 16 + mb * 16 + a;
            af[mb] = *reinterpret_cast<const float4*>(xs + r * 128 + ((c ^ swz(r)) * 16));
          }
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const int r = nb * 16 + a;
            bf[nb] = *reinterpret_cast<const float4*>(vs + r * 128 + ((c ^ swz(r)) * 16));
          }
#pragma unroll
          for (int mb = 0; mb < MW; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mb].x, bf[nb].x, acc[mb][nb], 0, 0, 0);
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mb].y, bf[nb].y, acc[mb][nb], 0, 0, 0);
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mb].z, bf[nb].z, acc[mb][nb], 0, 0, 0);
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mb].w, bf[nb].w, acc[mb][nb], 0, 0, 0);
            }
        }
      } else {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          uint4 af[MW], bf[NB];
          const int c = 4 * h + g;
#pragma unroll
          for (int mb = 0; mb < MW; ++mb) {
            const int r = w * MW * 16 + mb * 16 + a;
            af[mb] = *reinterpret_cast<const uint4*>(xs + r * 128 + ((c ^ swz(r)) * 16));
          }
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const int r = nb * 16 + a;
            bf[nb] = *reinterpret_cast<const uint4*>(vs + r * 128 + ((c ^ swz(r)) * 16));
          }
#pragma unroll
          for (int mb = 0; mb < MW; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
              acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(af[mb]), as_bf16x8(bf[nb]),
                                                                    acc[mb][nb], 0, 0, 0);
          if constexpr (SPLIT) {
            // second term: the same X fragments against lo
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
              const int r = nb * 16 + a;
              bf[nb] = *reinterpret_cast<const uint4*>(vs + VSB + r * 128 + ((c ^ swz(r)) * 16));
            }
#pragma unroll
            for (int mb = 0; mb < MW; ++mb)
#pragma unroll
              for (int nb = 0; nb < NB; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    as_bf16x8(af[mb]), as_bf16x8(bf[nb]), acc[mb][nb], 0, 0, 0);
          }
        }
      }
    };

    issue(0, 0);
    issue(1, 1);
    auto step = [&](int kk, auto B) __attribute__((always_inline)) {
      constexpr int b = decltype(B)::value;
      wait_vmcnt<DPS>();                     // this wave's DMA of step kk has landed
      if (dtail != 0 && kk == nk - 1) {
        fix_tail(b);
        wait_lgkm0();                        // the cleared chunks are written before the barrier
      }
      raw_barrier();                         // ... and every wave's; stage (b+2)%3 is free
      issue(kk + 2, (b + 2) % 3);
      if (kk < nk) compute(b);
    };
    for (int k = 0; k < nk; k += 3) {
      step(k, std::integral_constant<int, 0>{});
      step(k + 1, std::integral_constant<int, 1>{});
      step(k + 2, std::integral_constant<int, 2>{});
    }
    wait_vmcnt<0>();
    raw_barrier();                           // every DMA landed, every stage read

    if constexpr (PART) {
      // float32 partial of this split: ypart[split][row0 + lr][c]
      float* yp = ypart + ((int64_t)sb * yrows + row0) * Kp;
#pragma unroll
      for (int mb = 0; mb < MW; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int u = 0; u < 4; ++u)
            yp[(int64_t)(w * MW * 16 + mb * 16 + 4 * g + u) * Kp + nb * 16 + a] = acc[mb][nb][u];
    } else {
    // ---- Y tile -> LDS, layout [row/YR][Kp][YR]; rows [0, WGR/2) in st0, the
    // rest in st1.  Rows past the pass are written as zeros.
    const int64_t vrows = rows - row0;        // valid rows of this tile
#pragma unroll
    for (int mb = 0; mb < MW; ++mb) {
      const int lr = w * MW * 16 + mb * 16 + 4 * g;
      uint8_t* yh = lr < WGR / 2 ? st0 : st1;
      const int hr = lr & (WGR / 2 - 1);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = (lr + u < vrows) ? acc[mb][nb][u] : 0.f;
        if (DT == DT_F32) {
          *reinterpret_cast<float4*>(yh + ((hr >> 2) * Kp + nb * 16 + a) * 16) =
              make_float4(v[0], v[1], v[2], v[3]);
        } else {
          uint2 wv;
          wv.x = f32_to_bf16_bits(v[0]) | (f32_to_bf16_bits(v[1]) << 16);
          wv.y = f32_to_bf16_bits(v[2]) | (f32_to_bf16_bits(v[3]) << 16);
          *reinterpret_cast<uint2*>(yh + ((hr >> 3) * Kp + nb * 16 + a) * 16 + (hr & 7) * 2) = wv;
        }
      }
    }
    wait_lgkm0();
    raw_barrier();
    if (WANT_Y) {
      // coalesced copy of the tile to the staging buffer (same blocked layout)
      uint8_t* ydst = yb + row0 * Kp * EB;
      constexpr int HCH = YHB / 16;
      for (int sch = t; sch < 2 * HCH; sch += 256) {
        const uint8_t* src = sch < HCH ? st0 + sch * 16 : st1 + (sch - HCH) * 16;
        *reinterpret_cast<uint4*>(ydst + sch * 16) = *reinterpret_cast<const uint4*>(src);
      }
    }
    if constexpr (WANT_G) {
      // G += Y^T Y over the tile; wave w takes the column blocks nb = w + 4q.
      // The B fragments of those blocks are read by address (a register
      // array indexed by the wave number would live in scratch); blocks past
      // NB read block 0 and their products are never stored.
      constexpr int NCR = WGR / YR;                    // chunk rows of the tile
#pragma unroll
      for (int r0 = 0; r0 < NCR; r0 += 4) {
        const int rg = r0 + g;
        const uint8_t* yh = rg < NCR / 2 ? st0 : st1;
        const int hr = rg & (NCR / 2 - 1);
        const uint8_t* yrow = yh + (hr * Kp + a) * 16;
        if (DT == DT_F32) {
          float4 ya[NB], yw[NBG];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) ya[nb] = *reinterpret_cast<const float4*>(yrow + nb * 256);
#pragma unroll
          for (int q = 0; q < NBG; ++q) {
            const int nb = w + 4 * q;
            yw[q] = *reinterpret_cast<const float4*>(yrow + (nb < NB ? nb : 0) * 256);
          }
#pragma unroll
          for (int mb = 0; mb < NB; ++mb)
#pragma unroll
            for (int q = 0; q < NBG; ++q) {
              accg[mb][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ya[mb].x, yw[q].x, accg[mb][q], 0, 0, 0);
              accg[mb][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ya[mb].y, yw[q].y, accg[mb][q], 0, 0, 0);
              accg[mb][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ya[mb].z, yw[q].z, accg[mb][q], 0, 0, 0);
              accg[mb][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ya[mb].w, yw[q].w, accg[mb][q], 0, 0, 0);
            }
        } else {
          uint4 ya[NB], yw[NBG];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) ya[nb] = *reinterpret_cast<const uint4*>(yrow + nb * 256);
#pragma unroll
          for (int q = 0; q < NBG; ++q) {
            const int nb = w + 4 * q;
            yw[q] = *reinterpret_cast<const uint4*>(yrow + (nb < NB ? nb : 0) * 256);
          }
#pragma unroll
          for (int mb = 0; mb < NB; ++mb)
#pragma unroll
            for (int q = 0; q < NBG; ++q)
              accg[mb][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ya[mb]), as_bf16x8(yw[q]),
                                                                    accg[mb][q], 0, 0, 0);
        }
      }
    }
    }   // !PART
    // clear the accumulators for the next tile with a zero the compiler cannot
    // see through (a literal zero at the top of the tile makes the register
    // allocator rotate the accumulators through extra registers in the k-loop)
    const float zero = __uint_as_float(~keep);
#pragma unroll
    for (int mb = 0; mb < MW; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4_t{zero, zero, zero, zero};
    wait_lgkm0();
    raw_barrier();                           // the next tile's DMAs overwrite the Y tile
  }

  if constexpr (WANT_G) {
    float* gbase = gpart + (int64_t)tb * Kp * Kp;
#pragma unroll
    for (int mb = 0; mb < NB; ++mb)
#pragma unroll
      for (int q = 0; q < NBG; ++q) {
        const int nb = w + 4 * q;
        if (nb >= NB) continue;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          float* p = gbase + (int64_t)(mb * 16 + 4 * g + u) * Kp + nb * 16 + a;
          if (accumulate) *p += accg[mb][q][u];   // chunked passes only
          else *p = accg[mb][q][u];
        }
      }
  }
}

// ---------------------------------------------------------------------------
// Sum of the column-split partials of a short pass (k_xvd / k_xv in partial
// mode): workgroup w takes rows [16 w, 16 w + 16) of the pass; Y = sum over
// the splits in split order (float32), rows past the pass zero, rounded to
// bf16 for bf16/fp8 data; written to the Y staging buffer (blocked layout)
// when want_y; G_w = Y^T Y over the 16 rows (float32, rows in order) into
// gpart[w] when want_g (thread (i, j) of a 16 x 16 grid owns the NB x NB
// tile (i, j)).  Workgroups past the pass write zero G partials and zero Y
// rows: the grid covers the whole staging buffer (rows_cap rows), whose rows
// past the pass the X^T Y kernel reads in its last k-step.
// ---------------------------------------------------------------------------
constexpr int kYsumRows = 16;

template <int NB, int DT>
__global__ __launch_bounds__(256) void k_ysum(const float* __restrict__ ypart, int ksplit,
                                              int64_t yrows, int64_t rows, uint8_t* yb,
                                              float* gpart, int want_y, int want_g,
                                              int accumulate) {
  constexpr int Kp = NB * 16, RB = kYsumRows, LDY = Kp + 1, EPT = RB * Kp / 256;
  static_assert(DT == DT_F32 || DT == DT_BF16, "bf16 or f32 data");
  static_assert(EPT * 256 == RB * Kp, "elements per thread");
  __shared__ float ys[RB * LDY];
  const int t = threadIdx.x;
  const int64_t row0 = (int64_t)blockIdx.x * RB;
  const bool act = row0 < rows;             // uniform
  if (act) {
    // thread t sums elements t + 256 j over the splits, in split order; the
    // loads of 8 splits of all its elements are in flight together
    const int64_t ss = yrows * Kp;            // split stride
    const float* base = ypart + row0 * Kp;
    float sum[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) sum[j] = 0.f;
    for (int sp = 0; sp < ksplit; sp += 8) {
      float v[8][EPT];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int spu = sp + u < ksplit ? sp + u : ksplit - 1;
#pragma unroll
        for (int j = 0; j < EPT; ++j) v[u][j] = base[(int64_t)spu * ss + t + 256 * j];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int j = 0; j < EPT; ++j)
          if (sp + u < ksplit) sum[j] += v[u][j];
    }
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = t + 256 * j;
      const int r = e / Kp, c = e - r * Kp;
      const int64_t gr = row0 + r;
      float y = gr < rows ? sum[j] : 0.f;
      if constexpr (DT == DT_BF16) y = bf16_bits_to_f32(f32_to_bf16_bits(y));
      ys[r * LDY + c] = y;
      if (want_y) {
        if constexpr (DT == DT_F32)
          reinterpret_cast<float*>(yb)[((gr >> 2) * Kp + c) * 4 + (gr & 3)] = y;
        else
          reinterpret_cast<uint16_t*>(yb)[((gr >> 3) * Kp + c) * 8 + (gr & 7)] =
              (uint16_t)f32_to_bf16_bits(y);
      }
    }
  } else if (want_y) {
    // rows past the pass: the X^T Y kernel's last k-step reads them, as zeros
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = t + 256 * j;
      const int r = e / Kp, c = e - r * Kp;
      const int64_t gr = row0 + r;
      if constexpr (DT == DT_F32)
        reinterpret_cast<float*>(yb)[((gr >> 2) * Kp + c) * 4 + (gr & 3)] = 0.f;
      else
        reinterpret_cast<uint16_t*>(yb)[((gr >> 3) * Kp + c) * 8 + (gr & 7)] = 0;
    }
  }
  __syncthreads();
  if (!want_g) return;
  const int ti = t >> 4, tj = t & 15;
  float acc[NB][NB];
#pragma unroll
  for (int u = 0; u < NB; ++u)
#pragma unroll
    for (int v = 0; v < NB; ++v) acc[u][v] = 0.f;
  if (act) {
#pragma unroll 4
    for (int r = 0; r < RB; ++r) {
      float ra[NB], rb[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        ra[u] = ys[r * LDY + NB * ti + u];
        rb[u] = ys[r * LDY + NB * tj + u];
      }
#pragma unroll
      for (int u = 0; u < NB; ++u)
#pragma unroll
        for (int v = 0; v < NB; ++v) acc[u][v] = fmaf(ra[u], rb[v], acc[u][v]);
    }
  }
  float* gp = gpart + (int64_t)blockIdx.x * Kp * Kp;
#pragma unroll
  for (int u = 0; u < NB; ++u)
#pragma unroll
    for (int v = 0; v < NB; ++v) {
      float* q = gp + (int64_t)(NB * ti + u) * Kp + NB * tj + v;
      if (accumulate) *q += acc[u][v];
      else *q = acc[u][v];
    }
}

// ---------------------------------------------------------------------------
// Y = X V' of the power pass (bf16 data, Kp a multiple of 32, 256-row tiles,
// Y only).  The work split and LDS stages are those of k_xvd, but the DMA
// pipeline runs without a break over all (tile, k-step) pairs of the
// workgroup: the DMAs of the next tile's first steps are in flight while the
// current tile finishes, and the Y tile goes from the 32x32x16 accumulators
// straight to the blocked staging layout in global memory (no LDS copy, no
// barrier).  Element i of acc2[mb][nb] of lane (l32, hl) is row
// w * 64 + 32 mb + 8 (i / 4) + 4 hl + i % 4 of the tile, column 32 nb + l32;
// its four rows 8 j + 4 hl .. + 3 are one 8-byte piece of a 16-byte Y chunk,
// so each store writes 512 contiguous bytes per wavefront.
// ---------------------------------------------------------------------------
template <int NB>
__global__ __launch_bounds__(256, 1) void k_xvy(const uint8_t* x, int64_t n, int64_t d, int64_t ld,
                                                int64_t rstart, int64_t rows, const uint8_t* vop,
                                                int64_t dp, uint8_t* yb) {
  static_assert(NB % 2 == 0, "Kp a multiple of 32");
  constexpr int Kp = NB * 16, N2 = NB / 2, M2 = 2;
  constexpr int EB = 2, KS = 64, MW = 4, WGR = 64 * MW;
  constexpr int XSB = WGR * 128, VSB = Kp * 128, STB = XSB + VSB;
  constexpr int XI = WGR / 32, VBLK = Kp / 8, VI = (VBLK + 3) / 4, DPS = XI + VI;
  static_assert(2 * DPS < 64, "vmcnt range");
  __shared__ __attribute__((aligned(16))) uint8_t st[3 * STB];

  const int t = threadIdx.x, lane = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int l32 = lane & 31, hl = lane >> 5;
  const int64_t ntile = (rows + WGR - 1) / WGR;
  const int64_t mytiles = ntile > blockIdx.x ? (ntile - 1 - blockIdx.x) / gridDim.x + 1 : 0;
  const int nk = (int)((d + KS - 1) / KS);
  const int64_t nsteps = mytiles * nk;
  if (nsteps == 0) return;
  const int64_t klast = (int64_t)(nk - 1) * KS;
  const int64_t dtail = d % (16 / EB);

  // DMA sources, as in k_xvd
  const int p8 = lane & 7;
  int xc[XI];
#pragma unroll
  for (int j = 0; j < XI; ++j) {
    const int r = 8 * (w * XI + j) + (lane >> 3);
    xc[j] = (p8 ^ swz(r)) * (16 / EB);
  }
  const int64_t tstep = ((int64_t)gridDim.x * WGR) % n;
  int64_t xrow[XI];
  const uint8_t* xsrc[XI];
#pragma unroll
  for (int j = 0; j < XI; ++j) {
    const int r = 8 * (w * XI + j) + (lane >> 3);
    xrow[j] = (rstart + (int64_t)blockIdx.x * WGR + r) % n;
    xsrc[j] = x + xrow[j] * ld * EB;
  }
  const uint8_t* vsrc[VI];
  int vblk[VI];
#pragma unroll
  for (int j = 0; j < VI; ++j) {
    const int blk = (w * VI + j) % VBLK;
    const int r = 8 * blk + (lane >> 3);
    vblk[j] = blk;
    vsrc[j] = vop + (int64_t)r * dp * EB + (p8 ^ swz(r)) * 16;
  }
  // stage b of the ring (b is wavefront-uniform)
  auto stage = [&](int b) __attribute__((always_inline)) -> uint8_t* { return st + b * STB; };
  // issue side: next step iss = (tile ordinal, k-step ik); past the last
  // step the last one is loaded again (every wave issues the same count)
  int64_t iss = 0;
  int ik = 0;
  auto issue = [&](int b) __attribute__((always_inline)) {
    uint8_t* sb = stage(b);
    const int64_t k0 = iss < nsteps ? (int64_t)ik * KS : klast;
#pragma unroll
    for (int j = 0; j < XI; ++j) {
      const int64_t col = k0 + xc[j];
      dma16(xsrc[j] + (col < d ? col : 0) * EB, sb + (w * XI + j) * 1024);
    }
#pragma unroll
    for (int j = 0; j < VI; ++j) dma16(vsrc[j] + k0 * EB, sb + XSB + vblk[j] * 1024);
    if (iss < nsteps) {
      ++iss;
      if (++ik == nk) {
        if (iss < nsteps) {
          ik = 0;
#pragma unroll
          for (int j = 0; j < XI; ++j) {
            const int64_t nr = xrow[j] + tstep;
            xrow[j] = nr >= n ? nr - n : nr;
            xsrc[j] = x + xrow[j] * ld * EB;
          }
        } else {
          ik = nk - 1;
        }
      }
    }
  };
  auto fix_tail = [&](int b) __attribute__((always_inline)) {
    uint8_t* sb = stage(b);
#pragma unroll
    for (int j = 0; j < XI; ++j) {
      uint4* slot = reinterpret_cast<uint4*>(sb + (w * XI + j) * 1024 + lane * 16);
      *slot = and4(*slot, chunk_mask<EB>(klast + xc[j], d));
    }
  };

  f32x16_t acc2[M2][N2];
#pragma unroll
  for (int mb = 0; mb < M2; ++mb)
#pragma unroll
    for (int nb = 0; nb < N2; ++nb) acc2[mb][nb] = f32x16_t{};
  auto compute = [&](int b) __attribute__((always_inline)) {
    const uint8_t* xs = stage(b);
    const uint8_t* vs = xs + XSB;
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      uint4 af[M2], bf[N2];
      const int c = 2 * s4 + hl;
#pragma unroll
      for (int mb = 0; mb < M2; ++mb) {
        const int r = w * MW * 16 + mb * 32 + l32;
        af[mb] = *reinterpret_cast<const uint4*>(xs + r * 128 + ((c ^ swz(r)) * 16));
      }
#pragma unroll
      for (int nb = 0; nb < N2; ++nb) {
        const int r = nb * 32 + l32;
        bf[nb] = *reinterpret_cast<const uint4*>(vs + r * 128 + ((c ^ swz(r)) * 16));
      }
#pragma unroll
      for (int mb = 0; mb < M2; ++mb)
#pragma unroll
        for (int nb = 0; nb < N2; ++nb)
          acc2[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(af[mb]), as_bf16x8(bf[nb]),
                                                                 acc2[mb][nb], 0, 0, 0);
    }
  };
  // Y tile of tile ordinal ct from the accumulators; rows past the pass are zero
  const uint32_t keep = dp > 0 ? 0xFFFFFFFFu : 0u;   // all ones, opaque to the compiler
  auto store_y = [&](int64_t ct) __attribute__((always_inline)) {
    const int64_t row0 = ((int64_t)blockIdx.x + ct * gridDim.x) * WGR;
    const int64_t vrows = rows - row0;
    uint8_t* ybase = yb + (row0 / 8) * Kp * 16;
#pragma unroll
    for (int mb = 0; mb < M2; ++mb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int lr = w * MW * 16 + mb * 32 + 8 * j + 4 * hl;
#pragma unroll
        for (int nb = 0; nb < N2; ++nb) {
          float v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = (lr + u < vrows) ? acc2[mb][nb][4 * j + u] : 0.f;
          uint2 wv;
          wv.x = f32_to_bf16_bits(v[0]) | (f32_to_bf16_bits(v[1]) << 16);
          wv.y = f32_to_bf16_bits(v[2]) | (f32_to_bf16_bits(v[3]) << 16);
          *reinterpret_cast<uint2*>(ybase + ((lr >> 3) * Kp + nb * 32 + l32) * 16 + (lr & 7) * 2) = wv;
        }
      }
    // cleared with a zero the compiler cannot see through (see k_xvd)
    const float zero = __uint_as_float(~keep);
#pragma unroll
    for (int mb = 0; mb < M2; ++mb)
#pragma unroll
      for (int nb = 0; nb < N2; ++nb)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc2[mb][nb][i] = zero;
  };

  issue(0);
  issue(1);
  int b = 0;           // stage of the step being computed
  for (int64_t ct = 0; ct < mytiles; ++ct) {
    for (int kk = 0; kk < nk; ++kk) {
      wait_vmcnt<DPS>();                   // this wave's DMA of the step has landed
      if (dtail != 0 && kk == nk - 1) {
        fix_tail(b);
        wait_lgkm0();                      // the cleared chunks are written before the barrier
      }
      raw_barrier();                       // ... and every wave's; stage (b+2)%3 is free
      issue(b == 0 ? 2 : b - 1);
      compute(b);
      b = b == 2 ? 0 : b + 1;
    }
    store_y(ct);
  }
  wait_vmcnt<0>();
}

// ---------------------------------------------------------------------------
// Projection pass with a two-term operand (Alg. 1 steps 2-3; bf16 data, Kp a
// multiple of 32): V' = hi + lo with hi = bf16(V), lo = bf16(V - hi), so that
// the projected span is that of V to about 2^-16 instead of 2^-9.
// Y = X hi + X lo accumulates both products in one float32 accumulator
// (v_mfma_f32_32x32x16_bf16), is rounded to bf16, and G += Y^T Y is formed
// from the accumulators themselves: elements 0..7 and 8..15 of a lane's 32x32
// result block are rows {8 (e / 4) + 4 hl + e % 4} of one column, and serve
// as that lane's eight k-slots of two 32x32x16 products (the same rows for
// the A and the B operand), so Y never leaves the registers.
// Work split: persistent workgroups over 128-row tiles (each wave 32 rows),
// one DMA pipeline over all (tile, k-step) pairs as in k_xvy, three LDS
// stages of X (16 KB) + hi + lo (Kp x 128 bytes each).  The waves' G blocks
// are summed in LDS in wave order; one float32 partial per workgroup.
// ---------------------------------------------------------------------------
template <int NB>
__global__ __launch_bounds__(256, 1) void k_xvg(const uint8_t* x, int64_t n, int64_t d, int64_t ld,
                                                int64_t rstart, int64_t rows, const uint8_t* vop,
                                                int64_t dp, float* gpart, int accumulate) {
  static_assert(NB % 2 == 0, "Kp a multiple of 32");
  constexpr int Kp = NB * 16, N2 = NB / 2;
  constexpr int EB = 2, KS = 64, WGR = 128;
  constexpr int XSB = WGR * 128, VSB = Kp * 128, STB = XSB + 2 * VSB;
  constexpr int XI = WGR / 32, VBLK = Kp / 8, VI = (VBLK + 3) / 4, DPS = XI + 2 * VI;
  constexpr int NG = N2 * (N2 + 1) / 2;            // upper 32 x 32 blocks of G
  static_assert(2 * DPS < 64, "vmcnt range");
  static_assert(3 * STB <= 160 * 1024 && Kp * Kp * 4 <= 3 * STB, "LDS");
  __shared__ __attribute__((aligned(16))) uint8_t st[3 * STB];

  const int t = threadIdx.x, lane = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int l32 = lane & 31, hl = lane >> 5;
  const int64_t ntile = (rows + WGR - 1) / WGR;
  const int64_t mytiles = ntile > blockIdx.x ? (ntile - 1 - blockIdx.x) / gridDim.x + 1 : 0;
  const int nk = (int)((d + KS - 1) / KS);
  const int64_t nsteps = mytiles * nk;
  const int64_t klast = (int64_t)(nk - 1) * KS;
  const int64_t dtail = d % (16 / EB);

  // DMA sources, as in k_xvy
  const int p8 = lane & 7;
  int xc[XI];
#pragma unroll
  for (int j = 0; j < XI; ++j) {
    const int r = 8 * (w * XI + j) + (lane >> 3);
    xc[j] = (p8 ^ swz(r)) * (16 / EB);
  }
  const int64_t tstep = ((int64_t)gridDim.x * WGR) % n;
  int64_t xrow[XI];
  const uint8_t* xsrc[XI];
#pragma unroll
  for (int j = 0; j < XI; ++j) {
    const int r = 8 * (w * XI + j) + (lane >> 3);
    xrow[j] = (rstart + (int64_t)blockIdx.x * WGR + r) % n;
    xsrc[j] = x + xrow[j] * ld * EB;
  }
  const int64_t lo_off = (int64_t)Kp * dp * EB;     // lo follows hi
  const uint8_t* vsrc[VI];
  int vblk[VI];
#pragma unroll
  for (int j = 0; j < VI; ++j) {
    const int blk = (w * VI + j) % VBLK;
    const int r = 8 * blk + (lane >> 3);
    vblk[j] = blk;
    vsrc[j] = vop + (int64_t)r * dp * EB + (p8 ^ swz(r)) * 16;
  }
  auto stage = [&](int b) __attribute__((always_inline)) -> uint8_t* { return st + b * STB; };
  int64_t iss = 0;
  int ik = 0;
  auto issue = [&](int b) __attribute__((always_inline)) {
    uint8_t* sb = stage(b);
    const int64_t k0 = iss < nsteps ? (int64_t)ik * KS : klast;
#pragma unroll
    for (int j = 0; j < XI; ++j) {
      const int64_t col = k0 + xc[j];
      dma16(xsrc[j] + (col < d ? col : 0) * EB, sb + (w * XI + j) * 1024);
    }
#pragma unroll
    for (int j = 0; j < VI; ++j) {
      dma16(vsrc[j] + k0 * EB, sb + XSB + vblk[j] * 1024);
      dma16(vsrc[j] + lo_off + k0 * EB, sb + XSB + VSB + vblk[j] * 1024);
    }
    if (iss < nsteps) {
      ++iss;
      if (++ik == nk) {
        if (iss < nsteps) {
          ik = 0;
#pragma unroll
          for (int j = 0; j < XI; ++j) {
            const int64_t nr = xrow[j] + tstep;
            xrow[j] = nr >= n ? nr - n : nr;
            xsrc[j] = x + xrow[j] * ld * EB;
          }
        } else {
          ik = nk - 1;
        }
      }
    }
  };
  auto fix_tail = [&](int b) __attribute__((always_inline)) {
    uint8_t* sb = stage(b);
#pragma unroll
    for (int j = 0; j < XI; ++j) {
      uint4* slot = reinterpret_cast<uint4*>(sb + (w * XI + j) * 1024 + lane * 16);
      *slot = and4(*slot, chunk_mask<EB>(klast + xc[j], d));
    }
  };

  f32x16_t acc[N2], gacc[NG];
#pragma unroll
  for (int nb = 0; nb < N2; ++nb) acc[nb] = f32x16_t{};
#pragma unroll
  for (int i = 0; i < NG; ++i) gacc[i] = f32x16_t{};
  auto compute = [&](int b) __attribute__((always_inline)) {
    const uint8_t* xs = stage(b);
    const uint8_t* vh = xs + XSB;
    const uint8_t* vl = vh + VSB;
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int c = 2 * s4 + hl;
      const int r = w * 32 + l32;
      const uint4 af = *reinterpret_cast<const uint4*>(xs + r * 128 + ((c ^ swz(r)) * 16));
      uint4 bh[N2], bl[N2];
#pragma unroll
      for (int nb = 0; nb < N2; ++nb) {
        const int rv = nb * 32 + l32;
        bh[nb] = *reinterpret_cast<const uint4*>(vh + rv * 128 + ((c ^ swz(rv)) * 16));
        bl[nb] = *reinterpret_cast<const uint4*>(vl + rv * 128 + ((c ^ swz(rv)) * 16));
      }
#pragma unroll
      for (int nb = 0; nb < N2; ++nb)
        acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(af), as_bf16x8(bh[nb]), acc[nb],
                                                          0, 0, 0);
#pragma unroll
      for (int nb = 0; nb < N2; ++nb)
        acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(af), as_bf16x8(bl[nb]), acc[nb],
                                                          0, 0, 0);
    }
  };
  // G += Y^T Y of tile ordinal ct from the accumulators; rows past the pass are zero
  const uint32_t keep = dp > 0 ? 0xFFFFFFFFu : 0u;   // all ones, opaque to the compiler
  auto gram_tile = [&](int64_t ct) __attribute__((always_inline)) {
    const int64_t row0 = ((int64_t)blockIdx.x + ct * gridDim.x) * WGR;
    const int64_t vrows = rows - row0;
    uint4 yb[N2][2];
#pragma unroll
    for (int nb = 0; nb < N2; ++nb)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        uint32_t wv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e0 = 8 * h + 2 * q, e1 = e0 + 1;
          const int r0 = w * 32 + 8 * (e0 / 4) + 4 * hl + e0 % 4;
          const int r1 = w * 32 + 8 * (e1 / 4) + 4 * hl + e1 % 4;
          const float v0 = r0 < vrows ? acc[nb][e0] : 0.f;
          const float v1 = r1 < vrows ? acc[nb][e1] : 0.f;
          wv[q] = f32_to_bf16_bits(v0) | (f32_to_bf16_bits(v1) << 16);
        }
        yb[nb][h] = make_uint4(wv[0], wv[1], wv[2], wv[3]);
      }
    int idx = 0;
#pragma unroll
    for (int na = 0; na < N2; ++na)
#pragma unroll
      for (int nb = na; nb < N2; ++nb) {
        gacc[idx] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(yb[na][0]),
                                                            as_bf16x8(yb[nb][0]), gacc[idx], 0, 0, 0);
        gacc[idx] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(yb[na][1]),
                                                            as_bf16x8(yb[nb][1]), gacc[idx], 0, 0, 0);
        ++idx;
      }
    // cleared with a zero the compiler cannot see through (see k_xvd)
    const float zero = __uint_as_float(~keep);
#pragma unroll
    for (int nb = 0; nb < N2; ++nb)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[nb][i] = zero;
  };

  if (nsteps > 0) {
    issue(0);
    issue(1);
    int b = 0;
    for (int64_t ct = 0; ct < mytiles; ++ct) {
      for (int kk = 0; kk < nk; ++kk) {
        wait_vmcnt<DPS>();
        if (dtail != 0 && kk == nk - 1) {
          fix_tail(b);
          wait_lgkm0();
        }
        raw_barrier();
        issue(b == 0 ? 2 : b - 1);
        compute(b);
        b = b == 2 ? 0 : b + 1;
      }
      gram_tile(ct);
    }
  }
  wait_vmcnt<0>();
  raw_barrier();
  // sum the waves' G blocks in LDS, wave 0 first; element e of block (na, nb)
  // of lane (l32, hl) is G[32 na + 8 (e / 4) + 4 hl + e % 4][32 nb + l32]
  float* gl = reinterpret_cast<float*>(st);
#pragma unroll
  for (int ww = 0; ww < 4; ++ww) {
    if (w == ww) {
      int idx = 0;
#pragma unroll
      for (int na = 0; na < N2; ++na)
#pragma unroll
        for (int nb = na; nb < N2; ++nb) {
#pragma unroll
          for (int e = 0; e < 16; ++e) {
            const int i = 32 * na + 8 * (e / 4) + 4 * hl + e % 4, c = 32 * nb + l32;
            gl[i * Kp + c] = (ww == 0 ? 0.f : gl[i * Kp + c]) + gacc[idx][e];
          }
          ++idx;
        }
    }
    __syncthreads();
  }
  // the reduction reads the entries i <= c of every partial; chunked passes
  // add their chunks in order
  float* gp = gpart + (int64_t)blockIdx.x * Kp * Kp;
  for (int e = t; e < Kp * Kp; e += 256) {
    const int i = e / Kp, c = e % Kp;
    const float v = (i / 32 <= c / 32) ? gl[e] : 0.f;
    gp[e] = accumulate ? gp[e] + v : v;
  }
}

// Block id -> (tile, split).  Block b runs on XCD b mod 8; XCD x takes the
// contiguous run of (split, tile) pairs [x*per, (x+1)*per) in split-major
// order, so the tiles of one row split (which all read the same rows of Y)
// share that XCD's L2.  Blocks past the last pair return at once.
__device__ inline bool xty_tile_split(int ntiles, int nsplit, int& tile, int& split) {
  const int b = blockIdx.x;
  const int total = ntiles * nsplit;
  const int per = (total + 7) / 8;
  const int p = (b & 7) * per + (b >> 3);
  if ((b >> 3) >= per || p >= total) return false;
  split = p / ntiles;
  tile = p % ntiles;
  return true;
}

// ---------------------------------------------------------------------------
// Z partials, Z = X^T Y.  Workgroup (tile t, split s): the 256 columns
// [256t, 256t+256) of X (64 per wave) against all Kp columns of Y over the
// rows of split s, i.e. rows [s*rps, min(rows, (s+1)*rps)); k-step = 32 rows
// (16 for f32).  Output: part[t][s][Kp][256] float32; or, when the pass has
// a single row split and a single chunk (zd not null), Z itself:
// zd[j][c] = float(double(sum) * s_j) for j < d, c < K (s_j = 1 unless fp8),
// the value the fixed-order reduction of one partial would give.
// Each k-step's X rows (whole 512-byte row segments for bf16) and Y chunks go
// straight to LDS with global_load_lds into four LDS stages, three of them in
// flight while the MFMAs consume the fourth:
//   step kk: wait for this wave's DMA of step kk -> barrier -> DMA of step
//            kk+3 into the stage freed by step kk-1 -> MFMAs on stage kk.
// No masking is needed: columns past d only feed rows of Z that are never
// read; rows past the pass exist only in the last split, where the Y rows
// (written by the Y = X V' kernel) are zero.
// ---------------------------------------------------------------------------
template <int NB, int DT>
__global__ __launch_bounds__(256, 1) void k_xtyd(const uint8_t* x, int64_t n, int64_t d, int64_t ld,
                                                 int64_t rstart, int64_t rows, int64_t rps,
                                                 const uint8_t* yb, float* part, int ntiles,
                                                 int nsplit, int accumulate, float* zd, int K,
                                                 const float* zscale, int* status) {
  constexpr int Kp = NB * 16;
  constexpr int TC = 256;
  constexpr int EB = DT == DT_F32 ? 4 : DT == DT_BF16 ? 2 : 1;   // bytes per X element
  constexpr int YB = DT == DT_F32 ? 4 : 2;                        // bytes per Y element
  constexpr int KS = DT == DT_F32 ? 16 : 32;                      // rows per k-step
  constexpr int YR = 16 / YB;                                     // rows per Y chunk (8 or 4)
  constexpr int XRB = TC * EB;                                    // bytes per X row of a tile
  constexpr int XCPR = XRB / 16;                                  // chunks per X row
  constexpr int XSTB = KS * XRB;                                  // X bytes per stage
  constexpr int YSTB = KS * Kp * YB;                              // Y bytes per stage
  constexpr int STB = XSTB + YSTB;
  constexpr int RPB = 1024 / XRB;                                 // X rows per 1 KB DMA block
  constexpr int LPR = 64 / RPB;                                   // lanes per X row
  constexpr int XI = XSTB / 1024 / 4;                             // X DMAs per wave per step
  constexpr int YBLK = YSTB / 1024;                               // 1 KB blocks of a Y stage
  constexpr int YI = (YBLK + 3) / 4;                              // Y DMAs per wave per step
  constexpr int DPS = XI + YI;
  static_assert(XI * 4 * 1024 == XSTB && LPR == XCPR, "stage shape");
  static_assert(3 * DPS < 64, "vmcnt range");
  __shared__ __attribute__((aligned(16))) uint8_t st0[STB];
  __shared__ __attribute__((aligned(16))) uint8_t st1[STB];
  __shared__ __attribute__((aligned(16))) uint8_t st2[STB];
  __shared__ __attribute__((aligned(16))) uint8_t st3[STB];

  const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int a = lane & 15, g = lane >> 4;
  int tile, split;
  if (!xty_tile_split(ntiles, nsplit, tile, split)) return;
  const int64_t rbeg = (int64_t)split * rps;
  const int64_t rend = rbeg + rps < rows ? rbeg + rps : rows;
  const int64_t c0 = (int64_t)tile * TC;

  // X swizzle: chunk c of row r sits at slot c ^ xswz(r), so that the 4 lane
  // groups of a fragment read (rows 8 apart; 4 apart for f32) fall on
  // different banks
  auto xswz = [](int r) -> int {
    if (DT == DT_F32) return ((r >> 2) & 3) << 4;
    if (DT == DT_BF16) return ((r >> 3) & 3) << 3;
    return ((r >> 3) & 3) << 2;
  };

  // DMA sources.  X block j of wave w covers stage rows RPB (w XI + j) ..;
  // lane -> row RPB (w XI + j) + lane / LPR, slot lane % LPR holding chunk
  // slot ^ xswz(row).  Data rows advance by KS mod n per step.
  const int64_t ksn = KS % n;
  const uint8_t* xcp[XI];
  int64_t xrow[XI];
#pragma unroll
  for (int j = 0; j < XI; ++j) {
    const int r = RPB * (wave * XI + j) + lane / LPR;
    const int c = (lane % LPR) ^ xswz(r);
    const int64_t col = c0 + c * (16 / EB);
    xcp[j] = x + (col < d ? col : 0) * EB;
    xrow[j] = (rstart + rbeg + r) % n;
  }
  int yblk[YI];
#pragma unroll
  for (int j = 0; j < YI; ++j) yblk[j] = (wave * YI + j) % YBLK;

  const int64_t nk = rend > rbeg ? (rend - rbeg + KS - 1) / KS : 0;
  const int64_t llast = nk > 0 ? rbeg + (nk - 1) * KS : 0;

  auto stage = [&](int b) __attribute__((always_inline)) -> uint8_t* {
    return b == 0 ? st0 : (b == 1 ? st1 : (b == 2 ? st2 : st3));
  };
  // DMA of the step at pass row li into stage b (Y rows clamped to the last step)
  auto issue = [&](int64_t li, int b) __attribute__((always_inline)) {
    uint8_t* sb = stage(b);
#pragma unroll
    for (int j = 0; j < XI; ++j) {
      dma16(xcp[j] + xrow[j] * ld * EB, sb + (wave * XI + j) * 1024);
      const int64_t nr = xrow[j] + ksn;
      xrow[j] = nr >= n ? nr - n : nr;
    }
    const uint8_t* ysrc = yb + ((li < llast ? li : llast) / YR) * Kp * 16;
#pragma unroll
    for (int j = 0; j < YI; ++j) dma16(ysrc + yblk[j] * 1024 + lane * 16, sb + XSTB + yblk[j] * 1024);
  };

  f32x4_t acc[4][NB];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[v][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  const int cw = wave * 64 + 4 * a;   // this lane's first column inside the tile

  auto compute = [&](const uint8_t* xs) __attribute__((always_inline)) {
    const uint8_t* ys = xs + XSTB;
    if (DT == DT_F32) {
      // k-index of lane group g, MFMA s: row 4g + s of the step
      float4 bf[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        bf[nb] = *reinterpret_cast<const float4*>(ys + (g * Kp + nb * 16 + a) * 16);
      float4 in[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int r = 4 * g + s;
        const int c = cw >> 2;   // chunk of 4 floats
        in[s] = *reinterpret_cast<const float4*>(xs + (r * XCPR + (c ^ xswz(r))) * 16);
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float bs[4] = {bf[nb].x, bf[nb].y, bf[nb].z, bf[nb].w};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const float as[4] = {in[s].x, in[s].y, in[s].z, in[s].w};
#pragma unroll
          for (int v = 0; v < 4; ++v)
            acc[v][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(as[v], bs[s], acc[v][nb], 0, 0, 0);
        }
      }
    } else {
      // k-index of lane group g, element e: row 8g + e of the step
      uint4 bf[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        bf[nb] = *reinterpret_cast<const uint4*>(ys + (g * Kp + nb * 16 + a) * 16);
      uint2 in[8];
#pragma unroll
      for (int r8 = 0; r8 < 8; ++r8) {
        const int r = 8 * g + r8;
        if (DT == DT_FP8) {
          const int byte = cw;                       // 4 codes at column cw
          const int c = byte >> 4;
          const uint32_t w = *reinterpret_cast<const uint32_t*>(
              xs + (r * XCPR + (c ^ xswz(r))) * 16 + (byte & 15));
          in[r8] = fp8x4_to_bf16x4(w);
        } else {
          const int byte = cw * 2;                   // 4 bf16 at column cw
          const int c = byte >> 4;
          in[r8] = *reinterpret_cast<const uint2*>(xs + (r * XCPR + (c ^ xswz(r))) * 16 + (byte & 15));
        }
      }
      // in-register transpose: af[v] = column cw + v over rows 8g .. 8g+7
      uint4 af[4];
      af[0] = make_uint4((in[0].x & 0xFFFFu) | (in[1].x << 16), (in[2].x & 0xFFFFu) | (in[3].x << 16),
                         (in[4].x & 0xFFFFu) | (in[5].x << 16), (in[6].x & 0xFFFFu) | (in[7].x << 16));
      af[1] = make_uint4((in[0].x >> 16) | (in[1].x & 0xFFFF0000u), (in[2].x >> 16) | (in[3].x & 0xFFFF0000u),
                         (in[4].x >> 16) | (in[5].x & 0xFFFF0000u), (in[6].x >> 16) | (in[7].x & 0xFFFF0000u));
      af[2] = make_uint4((in[0].y & 0xFFFFu) | (in[1].y << 16), (in[2].y & 0xFFFFu) | (in[3].y << 16),
                         (in[4].y & 0xFFFFu) | (in[5].y << 16), (in[6].y & 0xFFFFu) | (in[7].y << 16));
      af[3] = make_uint4((in[0].y >> 16) | (in[1].y & 0xFFFF0000u), (in[2].y >> 16) | (in[3].y & 0xFFFF0000u),
                         (in[4].y >> 16) | (in[5].y & 0xFFFF0000u), (in[6].y >> 16) | (in[7].y & 0xFFFF0000u));
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[v][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(af[v]), as_bf16x8(bf[nb]),
                                                               acc[v][nb], 0, 0, 0);
    }
  };

  issue(rbeg, 0);
  issue(rbeg + KS, 1);
  issue(rbeg + 2 * KS, 2);
  auto step = [&](int64_t kk, auto B) __attribute__((always_inline)) {
    constexpr int b = decltype(B)::value;
    wait_vmcnt<2 * DPS>();                   // this wave's DMA of step kk has landed
    raw_barrier();                           // ... and every wave's; stage (b+3)%4 is free
    issue(rbeg + (kk + 3) * KS, (b + 3) % 4);
    if (kk < nk) compute(stage(b));
  };
  for (int64_t k = 0; k < nk; k += 4) {
    step(k, std::integral_constant<int, 0>{});
    step(k + 1, std::integral_constant<int, 1>{});
    step(k + 2, std::integral_constant<int, 2>{});
    step(k + 3, std::integral_constant<int, 3>{});
  }
  wait_vmcnt<0>();

  if (zd) {
    // lane (a, g): acc[v][nb][u] is column c0 + wave*64 + 16g + 4u + v of X,
    // column nb*16 + a of Y
    bool bad = false;
    const int64_t cb = c0 + wave * 64 + 16 * g;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int yc = nb * 16 + a;
      if (yc >= K) continue;
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t j = cb + 4 * u + v;
          if (j >= d) continue;
          const float zf = zscale ? (float)((double)acc[v][nb][u] * (double)zscale[j])
                                  : acc[v][nb][u];
          if (!isfinite(zf)) bad = true;
          zd[j * K + yc] = zf;
        }
    }
    if (bad) set_status(status, PPCA_ERR_NONFINITE);
    return;
  }
  if (c0 + wave * 64 < d) {
    // lane (j = a, g): acc[v][nb][u] is tile column wave*64 + 16g + 4u + v,
    // Y column nb*16 + a
    float* pbase = part + ((int64_t)tile * nsplit + split) * Kp * TC;
    const int64_t cl = wave * 64 + 16 * g;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      float* dst = pbase + (int64_t)(nb * 16 + a) * TC + cl;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float4 v = make_float4(acc[0][nb][u], acc[1][nb][u], acc[2][nb][u], acc[3][nb][u]);
        float4* p = reinterpret_cast<float4*>(dst + 4 * u);
        if (accumulate) {
          const float4 o = *p;
          *p = make_float4(o.x + v.x, o.y + v.y, o.z + v.z, o.w + v.w);
        } else {
          *p = v;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Fixed-order float64 reduction of the partials.
// Blocks [0, zblocks): Z[j][c] = s_j * sum_split part[j / 256][split][c][j mod 256]
//   (j < d, c < K; consecutive threads take consecutive j of one column c).
// Blocks [zblocks, ...): 64 consecutive elements (i, c) of G each; the 4
//   wavefronts sum the k_xv partials in 4 contiguous ranges, then wavefront 0
//   adds the 4 range sums in order: G[i][c] = sum_w gpart[w][i][c], i <= c,
//   mirrored.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce_zg(const float* __restrict__ part,
                                                   const float* __restrict__ gpart, int nsplit,
                                                   int ngpart, int Kp, int64_t d, int K,
                                                   const float* __restrict__ scale,
                                                   float* __restrict__ Z, double* __restrict__ G,
                                                   double* __restrict__ Gc, int zblocks,
                                                   int* status) {
  constexpr int TC = 256;
  __shared__ double gsum[4][64];
  bool bad = false;
  if ((int)blockIdx.x < zblocks) {
    const int64_t nz = d * K;
    const int64_t split_stride = (int64_t)Kp * TC;
    const int64_t tile_stride = (int64_t)nsplit * split_stride;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nz; e += (int64_t)zblocks * 256) {
      const int64_t c = e / d, j = e % d;
      const float* p = part + (j / TC) * tile_stride + c * TC + (j % TC);
      double s = 0.0;
      // splits in order, eight loads in flight
      int t = 0;
      for (; t + 8 <= nsplit; t += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(t + u) * split_stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += (double)v[u];
      }
      for (; t < nsplit; ++t) s += (double)p[(int64_t)t * split_stride];
      if (scale) s *= (double)scale[j];
      const float zf = (float)s;
      if (!isfinite(zf)) bad = true;
      Z[j * K + c] = zf;
    }
  } else {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t f = (int64_t)(blockIdx.x - zblocks) * 64 + lane;
    const int64_t i = f / K, c = f % K;
    const bool act = f < (int64_t)K * K && i <= c;
    const int per = (ngpart + 3) / 4;
    const int t0 = w * per, t1 = min(ngpart, t0 + per);
    double s = 0.0;
    if (act) {
      // partials in order, eight loads in flight
      const float* p = gpart + i * Kp + c;
      const int64_t st = (int64_t)Kp * Kp;
      int t = t0;
      for (; t + 8 <= t1; t += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(t + u) * st];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += (double)v[u];
      }
      for (; t < t1; ++t) s += (double)p[(int64_t)t * st];
    }
    gsum[w][lane] = s;
    __syncthreads();
    if (w == 0 && act) {
      const double g = ((gsum[0][lane] + gsum[1][lane]) + gsum[2][lane]) + gsum[3][lane];
      if (!isfinite(g)) bad = true;
      G[i * K + c] = g;
      G[c * K + i] = g;
      if (Gc) {
        Gc[i * K + c] = g;
        Gc[c * K + i] = g;
      }
    }
  }
  if (bad) set_status(status, PPCA_ERR_NONFINITE);
}

template <typename F>
hipError_t dispatch_nb(int Kp, F&& f) {
  switch (Kp / 16) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 3: return f(std::integral_constant<int, 3>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 5: return f(std::integral_constant<int, 5>{});
    case 6: return f(std::integral_constant<int, 6>{});
    case 7: return f(std::integral_constant<int, 7>{});
    case 8: return f(std::integral_constant<int, 8>{});
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int xty_cols(int Kp) {
  (void)Kp;
  return 256;
}

int xty_blocks_per_cu(int Kp) {
  (void)Kp;
  return 1;
}

int xty_tiles(int64_t d, int Kp) { return (int)cdiv(d, xty_cols(Kp)); }

// Row blocks per wave (MW) of k_xv: 4 (256-row tiles) when the pass is long
// enough to give every CU several tiles, else 1 (64-row tiles); float32 with
// K > 64 uses 2 (128-row tiles) so that the float32 Y tile fits in LDS.
constexpr int xv_wide_nb(int dt) { return dt == DT_F32 ? 4 : 8; }

static int xv_mw(int32_t dtype, int Kp, int64_t rows_cap) {
  if (rows_cap < (int64_t)kNumCU * 256) return 1;
  return Kp / 16 > xv_wide_nb(dtype) ? 2 : 4;
}

// Register stages of the fp8 Y = X V' pipeline: bytes of X in flight per CU
// grow with them, the register file bounds them (6 leaves every instance
// spill free with at least two stages in flight at each wait).
constexpr int xv_stages(int dt, int nb, int mw) { return 6; }

// Column splits of a short pass (64-row tiles): with few tiles the Y = X V'
// kernel runs on a few CUs, so the k-steps are split over up to 16
// workgroups per tile (at most 256 in all, every split at least one k-step)
// and a second kernel sums the float32 partials.  1 = no split.
// Row tiles of the column-split pass: 128 rows (two 16-row blocks per wave)
// when the rows are long (2048+ k-steps) and the data goes through the
// LDS-DMA kernel, else 64.  Each tile re-reads its split's slice of V' (for
// the two-term projection as many bytes as the tile's X), so taller tiles
// cut that traffic: measured at 6654 x 4M bf16 the two-term projection took
// 18.5 / 16.4 / 17.0 ms with 64 / 128 / 256-row tiles, the minibatch pass at
// 1024 x 15.1M 5.31 / 5.18 / 6.41 ms (256-row tiles leave too few
// workgroups).  Short rows keep 64-row tiles and more workgroups.
int split_rows(int32_t dtype, int64_t d) {
  const int64_t nk = cdiv(d, dtype == PPCA_BF16 ? 64 : 32);
  return (nk >= 2048 && dtype != PPCA_FP8_E4M3) ? 128 : 64;
}

int xv_ksplit(int32_t dtype, int Kp, int64_t d, int64_t rows_cap) {
  if (xv_mw(dtype, Kp, rows_cap) != 1) return 1;
  const int64_t ntile = cdiv(rows_cap, split_rows(dtype, d));
  if (ntile > 128) return 1;
  // columns per k-step: k_xvd 128 bytes of a row (f32 32, bf16 64), k_xv (fp8) 32
  const int64_t nk = cdiv(d, dtype == PPCA_BF16 ? 64 : 32);
  // long rows (d in the millions for bf16): up to 32 splits of at least 64
  // k-steps each, aiming at six workgroups per CU (measured at 1024 x 15.1M
  // bf16, 16 row tiles: 256 workgroups 4.6 TB/s, 512 5.8 TB/s, 1024 5.5 TB/s;
  // at 6654 x 1,048,576, 104 tiles, the two-term projection took 5.07 / 4.60
  // / 4.37 ms with 4 / 7 / 14 splits; at 6654 x 15.1M it reads 4.3 TB/s with
  // either split count); shorter rows keep one per CU and at most 16
  // splits, so the partial sums stay small beside X
  const bool long_rows = nk >= 2048;
  const int64_t cap = long_rows ? 32 : 16, per_cu = long_rows ? 6 : 1;
  int64_t target = std::min<int64_t>(cap, std::min<int64_t>(per_cu * kNumCU / ntile, nk));
  // long rows: a multiple of 8 splits, so that each split's tiles share an XCD
  if (long_rows && target >= 8) target -= target % 8;
  if (target < 2) return 1;
  const int64_t kper = cdiv(nk, target);
  return (int)cdiv(nk, kper);
}

int xvg_grid(int64_t rows_cap) {
  const int64_t tiles = cdiv(rows_cap, 128);
  return (int)(tiles < kNumCU ? tiles : kNumCU);
}

int xv_grid(int32_t dtype, int Kp, int64_t d, int64_t rows_cap) {
  // split short passes: one G partial per k_ysum workgroup (16 rows)
  if (xv_ksplit(dtype, Kp, d, rows_cap) > 1) return (int)cdiv(rows_cap, kYsumRows);
  const int64_t tiles = cdiv(rows_cap, 64 * xv_mw(dtype, Kp, rows_cap));
  return (int)(tiles < kNumCU ? tiles : kNumCU);
}

hipError_t launch_xv(const PassDesc& p, const StreamBufs& b, int64_t i0, int64_t rows,
                     bool want_y, bool want_g, bool accumulate, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  if (!want_y && !want_g) return hipErrorInvalidValue;
  const int64_t rstart = (p.r0 + i0) % p.n;
  const int mw = xv_mw(p.dtype, b.Kp, b.rows_cap);
  return dispatch_nb(b.Kp, [&](auto nbc) -> hipError_t {
    constexpr int NB = decltype(nbc)::value;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(b.ngpart), dim3(256), 0, s, (const uint8_t*)p.x, p.n, p.d,
                         p.ld, rstart, rows, (const uint8_t*)b.vop, b.dp, (uint8_t*)b.yb, b.gpart,
                         accumulate ? 1 : 0, (float*)nullptr, (int64_t)0);
    };
    // short pass with a column split: partial products, then their sum (Y of
    // fp8 data is rounded to bf16 like that of bf16 data)
    auto go_split = [&](auto dtc) {
      constexpr int DT = decltype(dtc)::value;
      const int srows = split_rows(p.dtype, p.d);
      const int64_t ntile = cdiv(rows, srows);
      const int64_t yrows = round_up(b.rows_cap, 64);
      // k_xv takes a (tile, split) grid, k_xvd a (split, tile) grid
      auto part = [&](auto kern, bool split_major) {
        const dim3 grid = split_major ? dim3(b.ksplit, ntile) : dim3(ntile, b.ksplit);
        hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, (const uint8_t*)p.x, p.n, p.d, p.ld,
                           rstart, rows, (const uint8_t*)b.vop, b.dp, (uint8_t*)nullptr,
                           (float*)nullptr, 0, b.ypart, yrows);
      };
      if constexpr (DT == DT_FP8)
        part(k_xv<NB, DT, 1, xv_stages(DT, NB, 1), false, false, true>, false);
      else if (srows == 128) part(k_xvd<NB, DT, 2, false, false, true>, true);
      else part(k_xvd<NB, DT, 1, false, false, true>, true);
      constexpr int DY = DT == DT_F32 ? DT_F32 : DT_BF16;
      hipLaunchKernelGGL((k_ysum<NB, DY>), dim3(b.ngpart), dim3(256), 0, s, b.ypart, b.ksplit,
                         yrows, rows, (uint8_t*)b.yb, b.gpart, want_y ? 1 : 0, want_g ? 1 : 0,
                         accumulate ? 1 : 0);
    };
    // projection of bf16 data with the two-term operand: short passes split
    // their columns (partial products of both terms, then k_ysum), longer
    // ones run k_xvg
    if (b.split) {
      if (p.dtype != PPCA_BF16 || !want_g || want_y) return hipErrorInvalidValue;
      if (b.ksplit > 1) {
        const int srows = split_rows(p.dtype, p.d);
        const int64_t ntile = cdiv(rows, srows);
        const int64_t yrows = round_up(b.rows_cap, 64);
        auto sp = [&](auto kern) {
          hipLaunchKernelGGL(kern, dim3(b.ksplit, ntile), dim3(256), 0, s, (const uint8_t*)p.x, p.n,
                             p.d, p.ld, rstart, rows, (const uint8_t*)b.vop, b.dp, (uint8_t*)nullptr,
                             (float*)nullptr, 0, b.ypart, yrows);
        };
        if (srows == 128) sp(k_xvd<NB, DT_BF16, 2, false, false, true, true>);
        else sp(k_xvd<NB, DT_BF16, 1, false, false, true, true>);
        hipLaunchKernelGGL((k_ysum<NB, DT_BF16>), dim3(b.ngpart), dim3(256), 0, s, b.ypart,
                           b.ksplit, yrows, rows, (uint8_t*)b.yb, b.gpart, 0, 1,
                           accumulate ? 1 : 0);
        return hipGetLastError();
      }
      if constexpr (NB % 2 == 0) {
        hipLaunchKernelGGL(k_xvg<NB>, dim3(b.ngpart), dim3(256), 0, s, (const uint8_t*)p.x, p.n,
                           p.d, p.ld, rstart, rows, (const uint8_t*)b.vop, b.dp, b.gpart,
                           accumulate ? 1 : 0);
        return hipGetLastError();
      }
      return hipErrorInvalidValue;
    }
    // bf16 / f32 data: LDS-DMA kernel; fp8 data: register-staged kernel
    auto by_mw = [&](auto dtc, auto yc, auto gc) {
      constexpr int DT = decltype(dtc)::value;
      constexpr bool WY = decltype(yc)::value, WG = decltype(gc)::value;
      if (mw == 1 && b.ksplit > 1) {
        go_split(dtc);
      } else if constexpr (DT == DT_FP8) {
        if (mw == 1) go(k_xv<NB, DT, 1, xv_stages(DT, NB, 1), WY, WG>);
        else go(k_xv<NB, DT, 4, xv_stages(DT, NB, 4), WY, WG>);
      } else {
        if (mw == 1) {
          go(k_xvd<NB, DT, 1, WY, WG>);
        } else if constexpr (DT == DT_BF16 && NB % 2 == 0 && WY && !WG) {
          hipLaunchKernelGGL(k_xvy<NB>, dim3(b.ngpart), dim3(256), 0, s, (const uint8_t*)p.x, p.n,
                             p.d, p.ld, rstart, rows, (const uint8_t*)b.vop, b.dp, (uint8_t*)b.yb);
        } else {
          if constexpr (NB > xv_wide_nb(DT)) go(k_xvd<NB, DT, 2, WY, WG>);
          else go(k_xvd<NB, DT, 4, WY, WG>);
        }
      }
    };
    auto by_dt = [&](auto yc, auto gc) {
      if (p.dtype == PPCA_F32) by_mw(std::integral_constant<int, DT_F32>{}, yc, gc);
      else if (p.dtype == PPCA_BF16) by_mw(std::integral_constant<int, DT_BF16>{}, yc, gc);
      else by_mw(std::integral_constant<int, DT_FP8>{}, yc, gc);
    };
    if (want_y && want_g) by_dt(std::true_type{}, std::true_type{});
    else if (want_y) by_dt(std::true_type{}, std::false_type{});
    else by_dt(std::false_type{}, std::true_type{});
    return hipGetLastError();
  });
}

hipError_t launch_xty(const PassDesc& p, const StreamBufs& b, int64_t i0, int64_t rows,
                      bool accumulate, float* Z, int K, int* status, hipStream_t s) {
  if (Z && (b.nsplit != 1 || accumulate)) return hipErrorInvalidValue;
  const float* zscale = p.dtype == PPCA_FP8_E4M3 ? p.col_scale : nullptr;
  if (rows <= 0) return hipSuccess;
  const int64_t rstart = (p.r0 + i0) % p.n;
  const int ntiles = xty_tiles(p.d, b.Kp);
  const int step = p.dtype == PPCA_F32 ? 16 : 32;
  const int64_t rps = round_up(cdiv(rows, b.nsplit), step);
  const int64_t grid = 8 * cdiv((int64_t)ntiles * b.nsplit, 8);
  return dispatch_nb(b.Kp, [&](auto nbc) -> hipError_t {
    constexpr int NB = decltype(nbc)::value;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, s, (const uint8_t*)p.x, p.n, p.d, p.ld,
                         rstart, rows, rps, (const uint8_t*)b.yb, b.part, ntiles, b.nsplit,
                         accumulate ? 1 : 0, Z, K, zscale, status);
    };
    if (p.dtype == PPCA_F32) go(k_xtyd<NB, DT_F32>);
    else if (p.dtype == PPCA_BF16) go(k_xtyd<NB, DT_BF16>);
    else go(k_xtyd<NB, DT_FP8>);
    return hipGetLastError();
  });
}

hipError_t launch_reduce_zg(const StreamBufs& b, int64_t d, int K, const float* col_scale,
                            float* Z, double* G, double* G_copy, bool gram_only, int* status,
                            hipStream_t s) {
  int64_t zb = gram_only ? 0 : cdiv(d * K, 256);
  if (zb > 2048) zb = 2048;
  const int64_t gb = G ? cdiv((int64_t)K * K, 64) : 0;
  if (zb + gb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_zg, dim3(zb + gb), dim3(256), 0, s, b.part, b.gpart, b.nsplit,
                     b.ngpart, b.Kp, d, K, col_scale, Z, G, G_copy, (int)zb, status);
  return hipGetLastError();
}

}  // namespace ppca
