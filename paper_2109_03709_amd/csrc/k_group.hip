// Grouped primed PCA: hundreds of independent problems (bf16 data, d <= 768,
// K = k + l <= 64) in a handful of launches per power iteration.
//
//   k_gpass     fused power / projection pass (Sec. 2.1; Alg. 1 steps 2-3) over
//               the work items of all problems: Y = X V', Y' = bf16(Y), then
//               Z += X^T Y' (power pass) or G += Y'^T Y' (projection pass; the
//               power iterations need no G).  X is read once per pass: the four
//               waves of a workgroup split the columns of a 16-row tile, each
//               wave's slice of X is staged in its own LDS buffers by DMA and
//               used for both products, and the partial Y of the waves is
//               summed through LDS.  All products run on 32x32x16 MFMAs (with
//               one wave per SIMD they sustain about 2.5 times the rate of the
//               16x16 shapes): Y over pairs of 16-row tiles (M = 32 rows),
//               the second products with K = the 16 rows of one tile.
//   k_greduce   fixed-order float64 sums of the item partials -> Z (f32), G (f64)
//   k_gcholqr2  CholeskyQR2 per problem (one workgroup, largest problems
//               launched first): new V, its bf16
//               operand, and B = V'^T V' after the last step
//   k_grr_h / k_grr_jacobi / k_grr_e
//               Rayleigh-Ritz per problem (Alg. 1 step 4): R = chol(B),
//               H = R^-T G R^-1 / n, Jacobi, E = V' R^-1 W[:, :k], signs.
//
// Shape classes of the fused pass (class width dc, waves per row tile WD,
// 64-column groups per wave CW):
//   dci 0: dc  64, WD 1, CW 1  (four independent row groups)
//   dci 1: dc 128, WD 1, CW 2  (four independent row groups; two waves per
//          row tile measured slower: their exchange costs as much as the
//          64 columns each wave reads)
//   dci 2: dc 256, WD 2, CW 2  (two row groups)
//   dci 3: dc 512, WD 4, CW 2
//   dci 4: dc 768, WD 4, CW 3
// combined with NB2 = Kp / 32 in 1..2 (K padded to 32): 10 code paths in one
// kernel.
//
// Partials: Z of item i, row group r: zpart[zoff + (r * Kp + c) * dc + j]
// (column c of Z, row j of Z); G of item i, wave w: gpart[goff + (w * Kp + c)
// * Kp + i] holds G_w[i][c] for i <= c (upper blocks; zero elsewhere).
#include "dense_dev.h"
#include "lds_dma.h"

namespace ppca {

// The class table above, the one definition that both the kernel (its wave
// layout) and the host plan (the number of partials per item) use.
constexpr int kClassWidth[kGroupClasses] = {64, 128, 256, 512, 768};
constexpr int kClassWD[kGroupClasses] = {1, 1, 2, 4, 4};   // waves sharing a row tile
constexpr int kClassCW[kGroupClasses] = {1, 2, 2, 2, 3};   // 64-column groups per wave
constexpr bool class_table_ok() {
  for (int i = 0; i < kGroupClasses; ++i)
    if (64 * kClassWD[i] * kClassCW[i] != kClassWidth[i] || 4 % kClassWD[i] != 0 ||
        (i > 0 && kClassWidth[i] <= kClassWidth[i - 1]))
      return false;
  return true;
}
static_assert(class_table_ok(), "class widths, wave split and order");

int group_class_width(int dci) { return kClassWidth[dci]; }
int group_row_groups(int dci) { return 4 / kClassWD[dci]; }
int group_dci(int64_t d) {
  for (int i = 0; i < kGroupClasses; ++i)
    if (d <= group_class_width(i)) return i;
  return -1;
}

namespace {

using namespace dma;
using dev::status_set;


template <int NB2, int DCI>
struct GCls {
  static constexpr int WD = kClassWD[DCI];                       // waves sharing a row tile
  static constexpr int CW = kClassCW[DCI];                       // 64-column groups per wave
  static constexpr int WR = 4 / WD;                              // row groups
  static constexpr int DW = 64 * CW;                             // columns per wave
  static constexpr int DC = WD * DW;                             // class width
  static constexpr int KP = 32 * NB2;                            // K padded to 32
  static constexpr int CPR = DW / 8;                             // 16-byte chunks per slice row
  static constexpr int XSB = 16 * DW * 2;                        // bytes of one stage
  static constexpr int DPS = XSB / 1024;                         // DMAs per stage
  static constexpr int NBT = NB2 * (NB2 + 1) / 2;                // upper blocks of G
  static constexpr int NGS = (NBT + WD - 1) / WD;                // G blocks per wave
  // X stages per wave: the same LDS for every class (24 KB per wave), so that
  // the narrow classes keep as many bytes in flight as the wide ones
  static constexpr int S = 4 * 16 * 192 * 2 / XSB;               // 12, 6 or 4
  static_assert((S - 1) * DPS < 64 && S >= 4 && S % 2 == 0, "stage ring");
  // LDS place of (row r, 16-byte chunk c) of a 16-row stage: physical row
  // prow(r), slot pch(r, c) (both involutions, so the DMA side uses them to
  // find the global chunk of a slot).  Two reads must be conflict-free:
  // the Y product reads one chunk of 16 rows (128-bit reads, 16 lanes a pass
  // over 16 units of 16 bytes), the Z product reads 8 chunks of rows r and
  // r + 4 (32-bit reads, 64 lanes a pass: the two rows' 128-byte windows must
  // be in different halves of the 256-byte bank window).  Rows of 128 CW
  // bytes: odd CW puts rows in alternate halves, so r and r + 4 swap
  // neighbours when bit 2 of r is set and the chunk swizzle takes r >> 1;
  // even CW keeps the rows and swizzles with the 4-bit r with bits 2 and 3
  // exchanged (bit 3 of the slot then differs between r and r + 4).
  static constexpr bool ODD = (CW & 1) != 0;
  __device__ static int prow(int r) { return ODD ? r ^ ((r >> 2) & 1) : r; }
  __device__ static int pch(int r, int c) {
    return ODD ? c ^ ((r >> 1) & 7) : c ^ ((r & 3) | ((r & 4) << 1) | ((r & 8) >> 1));
  }
};

constexpr int kGS = 4;                    // X stages per wave at the widest class
constexpr int kGStage = 16 * 192 * 2;     // bytes of one stage at the widest class
constexpr int kGExch = 4 * 2 * 4 * 64;    // f32 exchange slots [wave][nb][quarter][lane] (f32x4)
constexpr int kGExchB = 2 * 4 * 64;       // bf16 exchange slots [row group][nb][m][lane] (uint4)

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
// two floats to bf16, round to nearest even (v_cvt_pk_bf16_f32), lo in the low half
__device__ inline uint32_t pack2_bf16(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{lo, hi}, bf16x2_t));
}

// One work item (rows [r0, r0 + rows) of one problem) of class (NB2, DCI).
// Sub-tile t of row group rg covers item rows (t * WR + rg) * 16 .. + 15; the
// sub-tiles go in pairs (2 p, 2 p + 1), 32 rows, the M dimension of the
// 32x32x16 MFMAs of Y = X V'.  Lane l (l32 = l % 32, hl = l / 32) of a 32x32
// MFMA result holds element i at row 8 (i / 4) + 4 hl + i % 4 and column l32:
// the eight elements i = 8 m .. 8 m + 7 are rows of sub-tile m, and serve as
// this lane's eight k-slots (k = 8 hl + e <-> row 8 (e / 4) + 4 hl + e % 4 of
// sub-tile m) of the second products, Z += X^T Y' and G += Y'^T Y' on
// 32x32x16 MFMAs with K = the 16 rows of one sub-tile.
template <int NB2, int DCI, bool WZ>
__device__ __attribute__((always_inline)) inline void run_item(const GProb& P, const GItem& I,
                                                               uint8_t* xl, f32x4_t* exf,
                                                               uint4* exb,
                                                               float* zpart, float* gpart) {
  using C = GCls<NB2, DCI>;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rg = wave / C::WD, wd = wave % C::WD;
  const int l32 = lane & 31, hl = lane >> 5;
  const int c0 = wd * C::DW;
  const int64_t d = P.d, ld = P.ld, rows = I.rows, r0 = I.r0;
  const uint8_t* x = reinterpret_cast<const uint8_t*>(P.x);
  uint8_t* st = xl + wave * (kGS * kGStage);

  // operand fragments of this wave's column slice: k-substep s covers columns
  // c0 + 16 s .. + 15; lane (l32, hl) holds V' row 32 nb + l32, columns 8 hl ..
  uint4 vf[C::DW / 16][NB2];
#pragma unroll
  for (int s = 0; s < C::DW / 16; ++s)
#pragma unroll
    for (int nb = 0; nb < NB2; ++nb)
      vf[s][nb] = *reinterpret_cast<const uint4*>(P.vop + (int64_t)(32 * nb + l32) * C::DC + c0 +
                                                  16 * s + 8 * hl);
  // projection pass: the second term lo of the two-term operand, same layout
  constexpr int NLO = WZ ? 1 : C::DW / 16;
  uint4 vl[NLO][NB2];
  if constexpr (!WZ) {
#pragma unroll
    for (int s = 0; s < C::DW / 16; ++s)
#pragma unroll
      for (int nb = 0; nb < NB2; ++nb)
        vl[s][nb] = *reinterpret_cast<const uint4*>(P.vlo + (int64_t)(32 * nb + l32) * C::DC +
                                                    c0 + 16 * s + 8 * hl);
  }

  // DMA lanes: slot q = 64 j + lane of a stage is (physical row q / CPR,
  // slot q % CPR) and holds row r = prow(q / CPR) of the tile, 16-byte column
  // chunk pch(r, q % CPR) of the slice; chunks past d load column 0 (their
  // operand rows are zero).  voff: byte offset of lane's chunk j from its
  // tile's first row.
  auto drow = [&](int j) __attribute__((always_inline)) {
    return C::prow((64 * j + lane) / C::CPR);
  };
  auto dcol = [&](int j) __attribute__((always_inline)) {
    const int q = 64 * j + lane, r = C::prow(q / C::CPR), sl = q % C::CPR;
    const int64_t col = c0 + 8 * C::pch(r, sl);
    return (col < d ? col : 0) * 2;
  };
  uint32_t voff[C::DPS];
#pragma unroll
  for (int j = 0; j < C::DPS; ++j) voff[j] = (uint32_t)(drow(j) * ld * 2 + dcol(j));
  const int64_t srows = 16 * C::WR;
  const int64_t nsub = (rows + srows - 1) / srows;
  // DMA of sub-tile t into stage b (t clamped to the last sub-tile, rows past
  // the item clamped to its last row: every wave issues the same count).
  // Whole tiles take a scalar base and the 32-bit lane offsets.
  auto issue = [&](int64_t t, int b) __attribute__((always_inline)) {
    const int64_t tc = t < nsub ? t : nsub - 1;
    const int64_t lb = (tc * C::WR + rg) * 16;
    uint8_t* dst = st + b * C::XSB;
    if (lb + 16 <= rows) {
      const uint8_t* sb = x + (r0 + lb) * ld * 2;
#pragma unroll
      for (int j = 0; j < C::DPS; ++j) dma16s(sb, voff[j], dst + j * 1024);
    } else {
#pragma unroll
      for (int j = 0; j < C::DPS; ++j) {
        int64_t li = lb + drow(j);
        li = li < rows ? li : rows - 1;
        dma16(x + (r0 + li) * ld * 2 + dcol(j), dst + j * 1024);
      }
    }
  };

  // Z accumulators (Z pass: column group q, column parity v, block nb) or G
  // accumulators (G pass)
  constexpr int NZ = WZ ? C::CW : 0, NG = WZ ? 0 : C::NGS;
  f32x16_t zacc[NZ > 0 ? NZ : 1][2][NB2];
  f32x16_t gacc[NG > 0 ? NG : 1];
#pragma unroll
  for (int q = 0; q < NZ; ++q)
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int nb = 0; nb < NB2; ++nb) zacc[q][v][nb] = f32x16_t{};
#pragma unroll
  for (int i = 0; i < NG; ++i) gacc[i] = f32x16_t{};

  wait_vmcnt<0>();   // the operand fragments have landed before the DMA stream starts
  wait_lgkm0();      // LDS reads of the previous item are done before its stages refill
  // S - 2 sub-tiles are in flight ahead of the pair being used
#pragma unroll
  for (int b = 0; b < C::S - 2; ++b) issue(b, b);
  const int64_t npair = (nsub + 1) / 2;
  int bcur = 0;                 // stage of sub-tile 2 p
  for (int64_t p = 0; p < npair; ++p) {
    wait_vmcnt<(C::S - 4) * C::DPS>();   // the pair's sub-tiles have landed
    wait_lgkm0();                        // ... and the previous pair's have been read
    issue(2 * p + C::S - 2, bcur >= 2 ? bcur - 2 : bcur + C::S - 2);
    issue(2 * p + C::S - 1, bcur >= 1 ? bcur - 1 : bcur + C::S - 1);
    const uint8_t* xs0 = st + bcur * C::XSB;
    const uint8_t* xs1 = xs0 + C::XSB;
    bcur = bcur + 2 == C::S ? 0 : bcur + 2;

    // partial Y of the slice: lane row l32 of the pair (sub-tile l32 / 16),
    // k-substep s: chunk 2 s + hl
    f32x16_t ya[NB2];
#pragma unroll
    for (int nb = 0; nb < NB2; ++nb) ya[nb] = f32x16_t{};
    {
      const int rr = l32 & 15;
      const uint8_t* xrow = ((l32 >> 4) ? xs1 : xs0) + C::prow(rr) * C::CPR * 16;
#pragma unroll
      for (int s = 0; s < C::DW / 16; ++s) {
        const uint4 av = *reinterpret_cast<const uint4*>(xrow + C::pch(rr, 2 * s + hl) * 16);
#pragma unroll
        for (int nb = 0; nb < NB2; ++nb)
          ya[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(av), as_bf16x8(vf[s][nb]),
                                                           ya[nb], 0, 0, 0);
        if constexpr (!WZ) {
#pragma unroll
          for (int nb = 0; nb < NB2; ++nb)
            ya[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(av), as_bf16x8(vl[s][nb]),
                                                             ya[nb], 0, 0, 0);
        }
      }
    }
    // Y' = bf16(Y), rows past the item zeroed: yb[nb][m] holds this lane's
    // eight k-slots of sub-tile m (elements 8 m .. 8 m + 7 of ya[nb])
    uint4 yb[NB2][2];
    if constexpr (C::WD > 1) {
      // reduce-scatter: wave wd of the row group sums the values f = wd PS ..
      // wd PS + PS - 1 (f = 16 nb + i) over the group's waves in wave order,
      // rounds them and writes them to the row group's bf16 slots; then every
      // wave reads all of them.  The barriers also order the reuse of both
      // areas across pairs.
      constexpr int NV = 16 * NB2, PS = NV / C::WD;
      f32x4_t* mine = exf + wave * (NV / 4) * 64 + lane;
#pragma unroll
      for (int nb = 0; nb < NB2; ++nb)
#pragma unroll
        for (int qd = 0; qd < 4; ++qd)
          mine[(nb * 4 + qd) * 64] =
              f32x4_t{ya[nb][4 * qd], ya[nb][4 * qd + 1], ya[nb][4 * qd + 2], ya[nb][4 * qd + 3]};
      wait_lgkm0();
      raw_barrier();
      const f32x4_t* src = exf + rg * C::WD * (NV / 4) * 64 + wd * (PS / 4) * 64 + lane;
      float ys[PS];
#pragma unroll
      for (int u = 0; u < PS / 4; ++u) {
        f32x4_t y = src[u * 64];
#pragma unroll
        for (int j = 1; j < C::WD; ++j) y += src[(j * (NV / 4) + u) * 64];
#pragma unroll
        for (int c = 0; c < 4; ++c) ys[4 * u + c] = y[c];
      }
      uint32_t w[PS / 2];
#pragma unroll
      for (int v = 0; v < PS; v += 2) {
        float y2[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int i = (wd * PS + v + c) & 15, m = i >> 3, e = i & 7;
          const int64_t vr = rows - ((2 * p + m) * C::WR + rg) * 16;
          y2[c] = (8 * (e >> 2) + 4 * hl + (e & 3) < vr) ? ys[v + c] : 0.f;
        }
        w[v / 2] = pack2_bf16(y2[0], y2[1]);
      }
      uint32_t* eb = reinterpret_cast<uint32_t*>(exb + rg * (NV / 8) * 64);
      const int u0 = wd * (PS / 2);   // first dword of the part
      if constexpr (PS / 2 == 2) {
        *reinterpret_cast<uint2*>(eb + ((u0 / 4) * 64 + lane) * 4 + (u0 & 3)) =
            make_uint2(w[0], w[1]);
      } else {
#pragma unroll
        for (int s4 = 0; s4 < PS / 8; ++s4)
          *reinterpret_cast<uint4*>(eb + ((u0 / 4 + s4) * 64 + lane) * 4) =
              make_uint4(w[4 * s4], w[4 * s4 + 1], w[4 * s4 + 2], w[4 * s4 + 3]);
      }
      wait_lgkm0();
      raw_barrier();
#pragma unroll
      for (int nb = 0; nb < NB2; ++nb)
#pragma unroll
        for (int m = 0; m < 2; ++m) yb[nb][m] = exb[(rg * (NV / 8) + nb * 2 + m) * 64 + lane];
    } else {
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const int64_t vr = rows - ((2 * p + m) * C::WR + rg) * 16;
        float msk[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) msk[e] = (8 * (e / 4) + 4 * hl + e % 4 < vr) ? 1.f : 0.f;
#pragma unroll
        for (int nb = 0; nb < NB2; ++nb) {
          float y[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) y[e] = msk[e] != 0.f ? ya[nb][8 * m + e] : 0.f;
          yb[nb][m] = make_uint4(pack2_bf16(y[0], y[1]), pack2_bf16(y[2], y[3]),
                                 pack2_bf16(y[4], y[5]), pack2_bf16(y[6], y[7]));
        }
      }
    }
    // G += Y'^T Y' on the upper blocks (mb <= nb), dealt over the row group's waves
    if constexpr (!WZ) {
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int mb = 0; mb < NB2; ++mb)
#pragma unroll
          for (int nb = mb; nb < NB2; ++nb) {
            const int idx = mb * NB2 - mb * (mb - 1) / 2 + (nb - mb);
            if (idx % C::WD == wd)
              gacc[idx / C::WD] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                  as_bf16x8(yb[mb][m]), as_bf16x8(yb[nb][m]), gacc[idx / C::WD], 0, 0, 0);
          }
    }
    // Z += X^T Y': column group q (64 columns), lane l32 reads columns
    // 2 l32, 2 l32 + 1 of its eight k-slot rows of sub-tile m (4-byte reads):
    // A fragment v is column 2 l32 + v
    if constexpr (WZ) {
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const uint8_t* xs = m ? xs1 : xs0;
#pragma unroll
        for (int q = 0; q < C::CW; ++q) {
          uint32_t in[8];
          const int ch = 8 * q + (l32 >> 2);
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int row = 8 * (e / 4) + 4 * hl + e % 4;
            in[e] = *reinterpret_cast<const uint32_t*>(
                xs + (C::prow(row) * C::CPR + C::pch(row, ch)) * 16 + (l32 & 3) * 4);
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
            zacc[q][0][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                as_bf16x8(a0), as_bf16x8(yb[nb][m]), zacc[q][0][nb], 0, 0, 0);
            zacc[q][1][nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                as_bf16x8(a1), as_bf16x8(yb[nb][m]), zacc[q][1][nb], 0, 0, 0);
          }
        }
      }
    }
  }
  wait_vmcnt<0>();

  // partials.  Element i of lane (l32, hl) sits at M index mi = 8 (i / 4) +
  // 4 hl + i % 4.  Z: column c0 + 64 q + 2 mi + v of X, column 32 nb + l32 of Z.
  if constexpr (WZ) {
    float* zp = zpart + I.zoff + (int64_t)rg * C::KP * C::DC;
#pragma unroll
    for (int q = 0; q < C::CW; ++q)
#pragma unroll
      for (int nb = 0; nb < NB2; ++nb)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int mi = 8 * (i / 4) + 4 * hl + i % 4;
          *reinterpret_cast<float2*>(zp + (int64_t)(32 * nb + l32) * C::DC + c0 + 64 * q + 2 * mi) =
              make_float2(zacc[q][0][nb][i], zacc[q][1][nb][i]);
        }
  }
  // G: block (mb, nb), element i holds G[32 mb + mi][32 nb + l32]
  if constexpr (!WZ) {
    float* gp = gpart + I.goff + (int64_t)wave * C::KP * C::KP;
#pragma unroll
    for (int mb = 0; mb < NB2; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB2; ++nb) {
        f32x16_t v = f32x16_t{};
        if (mb <= nb) {
          const int idx = mb * NB2 - mb * (mb - 1) / 2 + (nb - mb);
          if (idx % C::WD == wd) v = gacc[idx / C::WD];
        }
#pragma unroll
        for (int i4 = 0; i4 < 4; ++i4)
          *reinterpret_cast<float4*>(gp + (32 * nb + l32) * C::KP + 32 * mb + 8 * i4 + 4 * hl) =
              make_float4(v[4 * i4], v[4 * i4 + 1], v[4 * i4 + 2], v[4 * i4 + 3]);
      }
  }
}

// Persistent fused pass: workgroup w takes items w, w + gridDim.x, ... (the
// items are sorted by size, largest first).  WZ: power pass (Z only);
// otherwise projection pass (G only).
template <bool WZ>
__global__ __launch_bounds__(256, 1) void k_gpass(const GProb* __restrict__ probs,
                                                  const GItem* __restrict__ items, int nitems,
                                                  float* zpart, float* gpart) {
  __shared__ __attribute__((aligned(16))) uint8_t xl[4 * kGS * kGStage];
  __shared__ f32x4_t exf[kGExch];
  __shared__ uint4 exb[kGExchB];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const GItem I = items[it];
    const GProb& P = probs[I.prob];
#define PPCA_GCASE(nb2, dci)                                             \
  case (dci) * 2 + (nb2) - 1:                                            \
    run_item<nb2, dci, WZ>(P, I, xl, exf, exb, zpart, gpart);            \
    break;
    switch (P.cls) {
      PPCA_GCASE(1, 0) PPCA_GCASE(2, 0) PPCA_GCASE(1, 1) PPCA_GCASE(2, 1)
      PPCA_GCASE(1, 2) PPCA_GCASE(2, 2) PPCA_GCASE(1, 3) PPCA_GCASE(2, 3)
      PPCA_GCASE(1, 4) PPCA_GCASE(2, 4)
      default: break;
    }
#undef PPCA_GCASE
  }
}

// ---------------------------------------------------------------------------
// Fixed-order float64 reduction.  Blocks of problem p: [blk0[p], blk0[p+1]);
// the first cdiv(d K, 256) of them (want_z) sum Z, one thread per element
// (column-major over the partial layout), the rest G (i <= c, mirrored).
// The partials of problem p are summed in item order, then row group / wave.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_greduce(const GProb* __restrict__ probs, int nprob,
                                                 const int* __restrict__ blk0,
                                                 const float* __restrict__ zpart,
                                                 const float* __restrict__ gpart, int want_z,
                                                 int* status) {
  const int bid = blockIdx.x;
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (blk0[mid] <= bid) lo = mid;
    else hi = mid - 1;
  }
  const GProb& P = probs[lo];
  const int b = bid - blk0[lo];
  const int64_t d = P.d;
  const int K = P.K, Kp = P.Kp, dc = P.dc;
  const int64_t zb = want_z ? (d * K + 255) / 256 : 0;
  const int t = threadIdx.x;
  if (b < zb) {
    const int64_t e = (int64_t)b * 256 + t;
    if (e >= d * K) return;
    const int c = (int)(e / d);
    const int64_t j = e - (int64_t)c * d;
    const int64_t stride = (int64_t)Kp * dc;
    const int np = P.nitem * P.wr;
    const float* zp = zpart + P.zbase + (int64_t)c * dc + j;
    double s = 0.0;
    int u = 0;
    for (; u + 8 <= np; u += 8) {
      float v[8];
#pragma unroll
      for (int w = 0; w < 8; ++w) v[w] = zp[(int64_t)(u + w) * stride];
#pragma unroll
      for (int w = 0; w < 8; ++w) s += (double)v[w];
    }
    for (; u < np; ++u) s += (double)zp[(int64_t)u * stride];
    if (!isfinite(s)) set_status(status, PPCA_ERR_NONFINITE);
    P.Z[j * K + c] = (float)s;
  } else {
    const int e = (int)(b - zb) * 256 + t;
    if (e >= K * K) return;
    const int i = e / K, c = e - i * K;
    if (i > c) return;
    const int64_t stride = (int64_t)Kp * Kp;
    const int np = P.nitem * 4;
    const float* gp = gpart + P.gbase + (int64_t)c * Kp + i;
    double s = 0.0;
    int u = 0;
    for (; u + 8 <= np; u += 8) {
      float v[8];
#pragma unroll
      for (int w = 0; w < 8; ++w) v[w] = gp[(int64_t)(u + w) * stride];
#pragma unroll
      for (int w = 0; w < 8; ++w) s += (double)v[w];
    }
    for (; u < np; ++u) s += (double)gp[(int64_t)u * stride];
    if (!isfinite(s)) set_status(status, PPCA_ERR_NONFINITE);
    P.G[i * K + c] = s;
    P.G[c * K + i] = s;
  }
}

// ---------------------------------------------------------------------------
// One-workgroup dense float64 helpers (256 threads, K <= 64).
// ---------------------------------------------------------------------------
constexpr int kGStg = 64;   // rows staged per step
constexpr int kGSp = 65;    // LDS row stride of a stage (odd: column reads spread banks)

// 64 x 64 stage of a rows x K block (zero outside): thread t holds elements
// t + 256 m (row e >> 6, column e & 63).  Loads use clamped indices and no
// branch, so that all 16 are in flight together.
template <typename Load>
__device__ inline void stage_load(Load load, int64_t r0, int64_t rows, int K, double (&reg)[16]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int e = t + 256 * m, rr = e >> 6, cc = e & 63;
    const int64_t r = r0 + rr;
    const double v = load(r < rows ? r : rows - 1, cc < K ? cc : K - 1);
    reg[m] = (r < rows && cc < K) ? v : 0.0;
  }
}
__device__ inline void stage_store(const double (&reg)[16], double* stg) {
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int e = threadIdx.x + 256 * m;
    stg[(e >> 6) * kGSp + (e & 63)] = reg[m];
  }
}

// out[i][c] = sum_r a(r, i) a(r, c) for a rows x K block on float64 MFMAs:
// the 16 x 16 blocks (ib <= jb) of the upper triangle are dealt to the four
// wavefronts (at most 3 each), which keep their accumulators across stages;
// each stage adds its 64 rows in order, 4 per MFMA.  out: global K x K, both
// triangles written.  stg: LDS [kGStg][kGSp]; the next stage is prefetched
// into registers while the current one is used.
template <typename Load>
__device__ inline void gram_wg(Load load, int64_t rows, int K, double* out, double* stg) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, l16 = lane & 15, g4 = lane >> 4;
  const int nbk = (K + 15) / 16, npair = nbk * (nbk + 1) / 2;
  int pib[3], pjb[3];
  dev::f64x4_t acc[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    int ib = 0, rem = wave + 4 * s;
    while (ib < nbk && rem >= nbk - ib) {
      rem -= nbk - ib;
      ++ib;
    }
    pib[s] = ib;
    pjb[s] = ib + rem;
    acc[s] = dev::f64x4_t{0.0, 0.0, 0.0, 0.0};
  }
  double nxt[16];
  stage_load(load, 0, rows, K, nxt);
  for (int64_t r0 = 0; r0 < rows; r0 += kGStg) {
    __syncthreads();
    stage_store(nxt, stg);
    __syncthreads();
    if (r0 + kGStg < rows) stage_load(load, r0 + kGStg, rows, K, nxt);
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      if (wave + 4 * s >= npair) break;
      const int ci = 16 * pib[s] + l16, cj = 16 * pjb[s] + l16;
#pragma unroll
      for (int kc = 0; kc < kGStg / 4; ++kc) {
        const double* row = stg + (4 * kc + g4) * kGSp;
        acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(row[ci], row[cj], acc[s], 0, 0, 0);
      }
    }
  }
  // acc[s][r]: row 16 ib + g4 + 4 r, column 16 jb + l16
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    if (wave + 4 * s >= npair) break;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * pib[s] + g4 + 4 * r, c = 16 * pjb[s] + l16;
      if (i < K && c < K && i <= c) {
        out[i * K + c] = acc[s][r];
        out[c * K + i] = acc[s][r];
      }
    }
  }
  __syncthreads();
}

// out(r, c) = sum_{p <= c} a(r, p) Rinv[p][c] for a rows x K block on float64
// MFMAs; Rl: LDS [64][64] copy of Rinv (zero below the diagonal and past K),
// stg: LDS [kGStg][kGSp].  Wavefront w takes the 16-row chunk w of every
// stage and all column blocks cb, summing the blocks p in 16 (cb + 1) in order.
template <typename Load, typename Store>
__device__ inline void trmm_wg(Load load, int64_t rows, int K, const double* Rinv, double* Rl,
                               double* stg, Store store) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, l16 = lane & 15, g4 = lane >> 4;
  const int nbk = (K + 15) / 16;
  __syncthreads();
  for (int e = t; e < 64 * 64; e += 256) {
    const int i = e >> 6, cc = e & 63;
    Rl[e] = (i < K && cc < K && i <= cc) ? Rinv[i * K + cc] : 0.0;
  }
  double nxt[16];
  stage_load(load, 0, rows, K, nxt);
  for (int64_t r0 = 0; r0 < rows; r0 += kGStg) {
    __syncthreads();
    stage_store(nxt, stg);
    __syncthreads();
    if (r0 + kGStg < rows) stage_load(load, r0 + kGStg, rows, K, nxt);
    const double* arow = stg + (16 * wave) * kGSp;
    for (int cb = 0; cb < nbk; ++cb) {
      dev::f64x4_t d = dev::f64x4_t{0.0, 0.0, 0.0, 0.0};
      for (int kb = 0; kb <= cb; ++kb)
        d = dev::mma16(d, [&](int i, int k) { return arow[i * kGSp + 16 * kb + k]; },
                       [&](int k, int j) { return Rl[(16 * kb + k) * 64 + 16 * cb + j]; });
      // d[r]: stage row 16 wave + g4 + 4 r, column 16 cb + l16
      const int c = 16 * cb + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t rr = r0 + 16 * wave + g4 + 4 * r;
        if (rr < rows && c < K) store(rr, c, d[r]);
      }
    }
  }
  __syncthreads();
}

// two-term operand of one problem: vop[c][j] = hi = bf16(V[j][c]) and
// vlo[c][j] = lo = bf16(V[j][c] - hi) (V - hi is exact in float32; zero for
// j >= d or c >= K, up to Kp x dc), by one workgroup of 256 threads.  The
// power passes multiply by hi, the projection pass by hi + lo.
__device__ inline void write_operand(const GProb& P, const float* V) {
  const int64_t d = P.d;
  const int K = P.K, Kp = P.Kp, dc = P.dc;
  for (int e = threadIdx.x; e < Kp * dc; e += 256) {
    const int c = e / dc, j = e - c * dc;
    const bool in = j < d && c < K;
    const float v = in ? V[(int64_t)j * K + c] : 0.f;
    const uint32_t hi = f32_to_bf16_bits(v);
    P.vop[e] = (uint16_t)hi;
    P.vlo[e] = (uint16_t)f32_to_bf16_bits(v - bf16_bits_to_f32(hi));
  }
}

// V_eff entry of the projection pass: hi + lo of V[j][c], exact in float64
__device__ inline double veff_two_term(float v) {
  const uint32_t hi = f32_to_bf16_bits(v);
  const float h = bf16_bits_to_f32(hi);
  return (double)h + (double)bf16_bits_to_f32(f32_to_bf16_bits(v - h));
}

// the operand of problem blockIdx.x from its V as it stands
__global__ __launch_bounds__(256) void k_goperand(const GProb* __restrict__ probs) {
  const GProb& P = probs[blockIdx.x];
  write_operand(P, P.V);
}

// CholeskyQR2 of Z (or of V when from_v) for problem blockIdx.x: V = Q, the
// two-term operand of V (write_operand) and, with want_b (before the
// projection pass), B = V_eff^T V_eff with V_eff = hi + lo.
//
// The staging area and the R^-1 copy of the block products share one LDS
// array with the Cholesky (the phases are separated by barriers): 66 KB per
// workgroup.  Registers still allow one workgroup per CU; bounding the kernel
// to two per CU spills and measured slower, as the time of a call is the
// chain of its largest problems rather than the number of resident ones.
constexpr int kGCholLds = kGStg * kGSp + 64 * 64;
__global__ __launch_bounds__(256) void k_gcholqr2(const GProb* __restrict__ probs,
                                                     const int* __restrict__ order, int from_v,
                                                     int want_b, int* status) {
  static_assert(dev::chol_lds_doubles<kGroupMaxK>() <= kGCholLds, "Cholesky area");
  __shared__ double lds[kGCholLds];
  double* const stg = lds;
  double* const Rl = lds + kGStg * kGSp;
  const GProb& P = probs[order[blockIdx.x]];
  const int64_t d = P.d;
  const int K = P.K;
  const float* src = from_v ? P.V : P.Z;
  double* q1 = P.q1;
  float* V = P.V;
  gram_wg([&](int64_t r, int c) { return (double)src[r * K + c]; }, d, K, P.A, stg);
  dev::chol_inv_dev<kGroupMaxK>(P.A, K, P.R, P.Rinv, status, lds);
  __syncthreads();
  trmm_wg([&](int64_t r, int c) { return (double)src[r * K + c]; }, d, K, P.Rinv, Rl, stg,
          [&](int64_t r, int c, double v) { q1[r * K + c] = v; });
  gram_wg([&](int64_t r, int c) { return q1[r * K + c]; }, d, K, P.A, stg);
  dev::chol_inv_dev<kGroupMaxK>(P.A, K, P.R, P.Rinv, status, lds);
  __syncthreads();
  trmm_wg([&](int64_t r, int c) { return q1[r * K + c]; }, d, K, P.Rinv, Rl, stg,
          [&](int64_t r, int c, double v) { V[r * K + c] = (float)v; });
  // operand (V was written by this workgroup before the barrier above)
  write_operand(P, V);
  if (want_b)
    gram_wg([&](int64_t r, int c) { return veff_two_term(V[r * K + c]); }, d, K, P.B, stg);
}

// Rayleigh-Ritz, part 1: R = chol(B), T = G R^-1, H = (R^-T T) / n.
__global__ __launch_bounds__(256) void k_grr_h(const GProb* __restrict__ probs,
                                               const int* __restrict__ order, int* status) {
  __shared__ double sh[3 * 64 * 64];
  double* const Rl = sh;
  double* const Gl = sh + 64 * 64;
  double* const Tl = sh + 2 * 64 * 64;
  const GProb& P = probs[order[blockIdx.x]];
  const int K = P.K, t = threadIdx.x;
  // the Cholesky works in the area of Gl and Tl, which are filled after it
  static_assert(dev::chol_lds_doubles<kGroupMaxK>() <= 2 * 64 * 64, "Cholesky area");
  dev::chol_inv_dev<kGroupMaxK>(P.B, K, P.R, P.Rinv, status, Gl);
  __syncthreads();
  for (int e = t; e < K * K; e += 256) {
    Rl[e] = P.Rinv[e];
    Gl[e] = P.G[e];
  }
  __syncthreads();
  for (int e = t; e < K * K; e += 256) {
    const int i = e / K, j = e - i * K;
    double s = 0.0;
    for (int p = 0; p < K; ++p) s = fma(Gl[i * K + p], Rl[p * K + j], s);
    Tl[e] = s;
  }
  __syncthreads();
  const double inv_n = 1.0 / (double)P.n;
  for (int e = t; e < K * K; e += 256) {
    const int i = e / K, j = e - i * K;
    double s = 0.0;
    for (int p = 0; p < K; ++p) s = fma(Rl[p * K + i], Tl[p * K + j], s);
    P.H[e] = inv_n * s;
  }
}

// Rayleigh-Ritz, part 2: Jacobi on H, one workgroup per problem holding all of W.
__global__ __launch_bounds__(1024) void k_grr_jacobi(const GProb* __restrict__ probs,
                                                     const int* __restrict__ order,
                                                     int max_sweeps, int* status) {
  const GProb& P = probs[order[blockIdx.x]];
  dev::jacobi_dev<kGroupMaxK, kGroupMaxK>(P.H, P.K, P.W, P.ev, max_sweeps, status, 0);
}

// Rayleigh-Ritz, part 3: M = R^-1 W[:, :k], E = V_eff M (V_eff = hi + lo of V),
// column signs (largest |.| positive, lowest row on ties), evals = theta[:k].
__global__ __launch_bounds__(256) void k_grr_e(const GProb* __restrict__ probs,
                                               const int* __restrict__ order, int* status) {
  __shared__ double Ml[64 * 64];
  __shared__ float bv[256];
  __shared__ int bi[256];
  __shared__ int flip[64];
  const GProb& P = probs[order[blockIdx.x]];
  const int K = P.K, k = P.k, t = threadIdx.x;
  const int64_t d = P.d;
  if (t < k) P.evals[t] = P.ev[t];
  if (P.E == nullptr) return;
  for (int e = t; e < K * k; e += 256) {
    const int i = e / k, j = e - i * k;
    double s = 0.0;
    for (int p = 0; p < K; ++p) s = fma(P.Rinv[i * K + p], P.W[p * K + j], s);
    Ml[e] = s;
  }
  __syncthreads();
  float* E = P.E;
  const float* V = P.V;
  for (int64_t e = t; e < d * k; e += 256) {
    const int64_t j = e / k;
    const int c = (int)(e - j * k);
    double s = 0.0;
    for (int p = 0; p < K; ++p) s = fma(veff_two_term(V[j * K + p]), Ml[p * k + c], s);
    E[e] = (float)s;
  }
  __syncthreads();
  // thread (c, g): rows g, g + ng, ... of column c
  const int ng = 256 / k;
  const int c = t % k, g = t / k;
  float best = -1.f;
  int bidx = 0;
  if (g < ng)
    for (int64_t j = g; j < d; j += ng) {
      const float v = fabsf(E[j * k + c]);
      if (v > best) {
        best = v;
        bidx = (int)j;
      }
    }
  bv[t] = best;
  bi[t] = bidx;
  __syncthreads();
  if (t < k) {
    float b = bv[t];
    int ix = bi[t];
    for (int h = 1; h < ng; ++h) {
      const float v = bv[h * k + t];
      const int i2 = bi[h * k + t];
      if (v > b || (v == b && i2 < ix)) {
        b = v;
        ix = i2;
      }
    }
    flip[t] = E[(int64_t)ix * k + t] < 0.f;
  }
  __syncthreads();
  for (int64_t e = t; e < d * k; e += 256) {
    const int cc = (int)(e % k);
    if (flip[cc]) E[e] = -E[e];
  }
}

}  // namespace

hipError_t launch_group_pass(const GProb* probs, const GItem* items, int nitems, int grid,
                             float* zpart, float* gpart, bool want_z, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (want_z)
    hipLaunchKernelGGL(k_gpass<true>, dim3(grid), dim3(256), 0, s, probs, items, nitems, zpart,
                       gpart);
  else
    hipLaunchKernelGGL(k_gpass<false>, dim3(grid), dim3(256), 0, s, probs, items, nitems, zpart,
                       gpart);
  return hipGetLastError();
}

hipError_t launch_group_reduce(const GProb* probs, int nprob, const int* blk0, int nblk,
                               const float* zpart, const float* gpart, bool want_z, int* status,
                               hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_greduce, dim3(nblk), dim3(256), 0, s, probs, nprob, blk0, zpart, gpart,
                     want_z ? 1 : 0, status);
  return hipGetLastError();
}

hipError_t launch_group_cholqr2(const GProb* probs, const int* order, int nprob, bool from_v,
                                bool want_b, int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_gcholqr2, dim3(nprob), dim3(256), 0, s, probs, order, from_v ? 1 : 0,
                     want_b ? 1 : 0, status);
  return hipGetLastError();
}

hipError_t launch_group_operand(const GProb* probs, int nprob, hipStream_t s) {
  hipLaunchKernelGGL(k_goperand, dim3(nprob), dim3(256), 0, s, probs);
  return hipGetLastError();
}

hipError_t launch_group_rr(const GProb* probs, const int* order, int nprob, int max_sweeps,
                           int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_grr_h, dim3(nprob), dim3(256), 0, s, probs, order, status);
  hipLaunchKernelGGL(k_grr_jacobi, dim3(nprob), dim3(1024), 0, s, probs, order, max_sweeps,
                     status);
  hipLaunchKernelGGL(k_grr_e, dim3(nprob), dim3(256), 0, s, probs, order, status);
  return hipGetLastError();
}

}  // namespace ppca
