// Streaming kernels of one pass over X (block power step, minibatch step and
// pPCA projection, Alg. 1 steps 2-3 and Sec. 2.1):
//
//   ppca_xv   : Y = X V'           (row panels of X, full d per workgroup)
//   ppca_xty  : [Z ; G] = [X | Y]^T Y over row splits (partial per split)
//   reduce_zg : fixed-order float64 sum of the partials -> Z (f32), G (f64)
//
// bf16 and fp8 data run on v_mfma_f32_16x16x32_bf16 (fp8 codes are widened
// to bf16 exactly); float32 data runs on v_mfma_f32_16x16x4_f32.  All
// accumulation inside a workgroup is float32; partials of different row
// splits are summed in float64 in a fixed order, so results are bitwise
// reproducible run to run.
//
// Layouts
//   X     row-major [n][ld] (element type per dtype); pass row i is data row
//         (r0 + i) mod n.
//   V'^T  operand [Kp][dp] (bf16 or f32), zero padded in both directions.
//   Y     "blocked" staging buffer so that the X^T Y kernel can read 8 (bf16)
//         or 4 (f32) consecutive rows of one Y column as a single 16-byte load:
//         bf16: yb[row/8][Kp][8], f32: yb[row/4][Kp][4].
//   part  [tile][split][Kp][256] float32: column c of tile t is column
//         t*256 + c of X (tiles 0..T-2) or column c of Y (last tile).
#include "ppca_common.h"

namespace ppca {

namespace {

__device__ inline bf16x8_t as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8_t, v); }

// widen 4 fp8 codes (one dword) to 4 bf16 (two dwords)
__device__ inline uint2 fp8x4_to_bf16x4(uint32_t w) {
  uint2 r;
  r.x = e4m3_to_bf16_bits(w & 0xFF) | (e4m3_to_bf16_bits((w >> 8) & 0xFF) << 16);
  r.y = e4m3_to_bf16_bits((w >> 16) & 0xFF) | (e4m3_to_bf16_bits(w >> 24) << 16);
  return r;
}

// 8 consecutive bf16 of a row starting at column `col` (zero beyond d).
template <bool FP8>
__device__ inline uint4 load_row8(const uint8_t* rowp, int64_t col, int64_t d) {
  uint4 v = make_uint4(0, 0, 0, 0);
  if (col + 8 <= d) {
    if (FP8) {
      const uint2 w = *reinterpret_cast<const uint2*>(rowp + col);
      const uint2 lo = fp8x4_to_bf16x4(w.x), hi = fp8x4_to_bf16x4(w.y);
      v = make_uint4(lo.x, lo.y, hi.x, hi.y);
    } else {
      v = *reinterpret_cast<const uint4*>(rowp + col * 2);
    }
  } else if (col < d) {
    uint32_t h[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      uint32_t b = 0;
      if (col + e < d) {
        b = FP8 ? e4m3_to_bf16_bits(rowp[col + e])
                : (uint32_t)reinterpret_cast<const uint16_t*>(rowp)[col + e];
      }
      h[e] = b;
    }
    v = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16),
                   h[6] | (h[7] << 16));
  }
  return v;
}

// 4 consecutive bf16 of a row starting at column `col` (zero beyond d).
template <bool FP8>
__device__ inline uint2 load_row4(const uint8_t* rowp, int64_t col, int64_t d) {
  uint2 v = make_uint2(0, 0);
  if (col + 4 <= d) {
    if (FP8) {
      v = fp8x4_to_bf16x4(*reinterpret_cast<const uint32_t*>(rowp + col));
    } else {
      v = *reinterpret_cast<const uint2*>(rowp + col * 2);
    }
  } else if (col < d) {
    uint32_t h[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      uint32_t b = 0;
      if (col + e < d) {
        b = FP8 ? e4m3_to_bf16_bits(rowp[col + e])
                : (uint32_t)reinterpret_cast<const uint16_t*>(rowp)[col + e];
      }
      h[e] = b;
    }
    v = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
  }
  return v;
}

__device__ inline float4 load_row4_f32(const float* rowp, int64_t col, int64_t d) {
  if (col + 4 <= d) return *reinterpret_cast<const float4*>(rowp + col);
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (col + 0 < d) v.x = rowp[col + 0];
  if (col + 1 < d) v.y = rowp[col + 1];
  if (col + 2 < d) v.z = rowp[col + 2];
  return v;
}

__device__ inline int64_t wrap_row(int64_t r, int64_t n) { return r < n ? r : r % n; }

// ---------------------------------------------------------------------------
// Y = X V'   (bf16 / fp8 data).  Workgroup: 4 waves x (MW x 16) rows.
// ---------------------------------------------------------------------------
template <int NB, int MW, bool FP8>
__global__ __launch_bounds__(256) void k_xv_b16(const uint8_t* __restrict__ x, int64_t n,
                                                int64_t d, int64_t ld, int64_t rstart,
                                                int64_t rows, const uint16_t* __restrict__ vop,
                                                int64_t dp, uint16_t* __restrict__ yb) {
  constexpr int ES = FP8 ? 1 : 2;
  constexpr int Kp = NB * 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int a = lane & 15, g = lane >> 4;
  const int64_t li0 = (int64_t)blockIdx.x * (4 * MW * 16) + wave * (MW * 16);

  const uint8_t* rowp[MW];
  bool rv[MW];
#pragma unroll
  for (int mb = 0; mb < MW; ++mb) {
    const int64_t li = li0 + mb * 16 + a;
    rv[mb] = li < rows;
    const int64_t r = rv[mb] ? (rstart + li) % n : 0;
    rowp[mb] = x + r * ld * ES;
  }
  const uint16_t* vp = vop + (int64_t)a * dp + 8 * g;

  f32x4_t acc[MW][NB];
#pragma unroll
  for (int mb = 0; mb < MW; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  uint4 an[MW], bn[NB];
#pragma unroll
  for (int mb = 0; mb < MW; ++mb)
    an[mb] = rv[mb] ? load_row8<FP8>(rowp[mb], 8 * g, d) : make_uint4(0, 0, 0, 0);
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
    bn[nb] = *reinterpret_cast<const uint4*>(vp + (int64_t)nb * 16 * dp);

  for (int64_t k0 = 0; k0 < d; k0 += 32) {
    uint4 ac[MW], bc[NB];
#pragma unroll
    for (int mb = 0; mb < MW; ++mb) ac[mb] = an[mb];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) bc[nb] = bn[nb];
    const int64_t kn = k0 + 32;
    if (kn < d) {
#pragma unroll
      for (int mb = 0; mb < MW; ++mb)
        an[mb] = rv[mb] ? load_row8<FP8>(rowp[mb], kn + 8 * g, d) : make_uint4(0, 0, 0, 0);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        bn[nb] = *reinterpret_cast<const uint4*>(vp + (int64_t)nb * 16 * dp + kn);
    }
#pragma unroll
    for (int mb = 0; mb < MW; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ac[mb]),
                                                              as_bf16x8(bc[nb]),
                                                              acc[mb][nb], 0, 0, 0);
  }

  // D[i][j]: lane (j = a, g) holds rows 4g..4g+3 of each 16-row block.
#pragma unroll
  for (int mb = 0; mb < MW; ++mb) {
    const int64_t li = li0 + mb * 16 + 4 * g;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      uint2 w;
      w.x = f32_to_bf16_bits(acc[mb][nb][0]) | (f32_to_bf16_bits(acc[mb][nb][1]) << 16);
      w.y = f32_to_bf16_bits(acc[mb][nb][2]) | (f32_to_bf16_bits(acc[mb][nb][3]) << 16);
      uint16_t* dst = yb + (((li >> 3) * Kp + nb * 16 + a) << 3) + (li & 7);
      *reinterpret_cast<uint2*>(dst) = w;
    }
  }
}

// ---------------------------------------------------------------------------
// Y = X V'   (float32 data), v_mfma_f32_16x16x4_f32.
// ---------------------------------------------------------------------------
template <int NB, int MW>
__global__ __launch_bounds__(256) void k_xv_f32(const float* __restrict__ x, int64_t n,
                                                int64_t d, int64_t ld, int64_t rstart,
                                                int64_t rows, const float* __restrict__ vop,
                                                int64_t dp, float* __restrict__ yb) {
  constexpr int Kp = NB * 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int a = lane & 15, g = lane >> 4;
  const int64_t li0 = (int64_t)blockIdx.x * (4 * MW * 16) + wave * (MW * 16);

  const float* rowp[MW];
  bool rv[MW];
#pragma unroll
  for (int mb = 0; mb < MW; ++mb) {
    const int64_t li = li0 + mb * 16 + a;
    rv[mb] = li < rows;
    const int64_t r = rv[mb] ? (rstart + li) % n : 0;
    rowp[mb] = x + r * ld;
  }
  const float* vp = vop + (int64_t)a * dp + 4 * g;

  f32x4_t acc[MW][NB];
#pragma unroll
  for (int mb = 0; mb < MW; ++mb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  float4 an[MW], bn[NB];
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
  for (int mb = 0; mb < MW; ++mb) an[mb] = rv[mb] ? load_row4_f32(rowp[mb], 4 * g, d) : z4;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
    bn[nb] = *reinterpret_cast<const float4*>(vp + (int64_t)nb * 16 * dp);

  for (int64_t k0 = 0; k0 < d; k0 += 16) {
    float4 ac[MW], bc[NB];
#pragma unroll
    for (int mb = 0; mb < MW; ++mb) ac[mb] = an[mb];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) bc[nb] = bn[nb];
    const int64_t kn = k0 + 16;
    if (kn < d) {
#pragma unroll
      for (int mb = 0; mb < MW; ++mb)
        an[mb] = rv[mb] ? load_row4_f32(rowp[mb], kn + 4 * g, d) : z4;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        bn[nb] = *reinterpret_cast<const float4*>(vp + (int64_t)nb * 16 * dp + kn);
    }
#pragma unroll
    for (int mb = 0; mb < MW; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ac[mb].x, bc[nb].x, acc[mb][nb], 0, 0, 0);
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ac[mb].y, bc[nb].y, acc[mb][nb], 0, 0, 0);
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ac[mb].z, bc[nb].z, acc[mb][nb], 0, 0, 0);
        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ac[mb].w, bc[nb].w, acc[mb][nb], 0, 0, 0);
      }
  }

#pragma unroll
  for (int mb = 0; mb < MW; ++mb) {
    const int64_t li = li0 + mb * 16 + 4 * g;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      float* dst = yb + (((li >> 2) * Kp + nb * 16 + a) << 2);
      *reinterpret_cast<float4*>(dst) =
          make_float4(acc[mb][nb][0], acc[mb][nb][1], acc[mb][nb][2], acc[mb][nb][3]);
    }
  }
}

// block id -> (tile, split) so that all tiles of one row split run on the
// same XCD (block b is dispatched to XCD b mod 8) and share Y through its L2.
__device__ inline void xty_tile_split(int ntiles, int& tile, int& split) {
  const int b = blockIdx.x;
  const int xcd = b & 7, slot = b >> 3;
  tile = slot % ntiles;
  split = (slot / ntiles) * 8 + xcd;
}

__device__ inline void store_part(float* dst, const float4 v, bool acc) {
  if (acc) {
    const float4 o = *reinterpret_cast<const float4*>(dst);
    *reinterpret_cast<float4*>(dst) = make_float4(o.x + v.x, o.y + v.y, o.z + v.z, o.w + v.w);
  } else {
    *reinterpret_cast<float4*>(dst) = v;
  }
}

// ---------------------------------------------------------------------------
// [Z ; G] partials, bf16 / fp8 data.  Tile t < ntiles-1: 256 columns of X
// (64 per wave); tile ntiles-1: the Kp columns of Y (Gram).  Rows of split s:
// [s*rps, min(rows, (s+1)*rps)).
// ---------------------------------------------------------------------------
template <int NB, bool FP8>
__global__ __launch_bounds__(256) void k_xty_b16(const uint8_t* __restrict__ x, int64_t n,
                                                 int64_t d, int64_t ld, int64_t rstart,
                                                 int64_t rows, int64_t rps,
                                                 const uint16_t* __restrict__ yb,
                                                 float* __restrict__ part, int ntiles,
                                                 int nsplit, int tile_base, int accumulate) {
  constexpr int ES = FP8 ? 1 : 2;
  constexpr int Kp = NB * 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int a = lane & 15, g = lane >> 4;
  int tile, split;
  xty_tile_split(ntiles, tile, split);
  tile += tile_base;
  const int64_t rbeg = (int64_t)split * rps;
  const int64_t rend = rbeg + rps < rows ? rbeg + rps : rows;
  float* pbase = part + ((int64_t)(tile - tile_base) * nsplit + split) * Kp * 256;
  const bool gram_tile = (tile == (int)((d + 255) / 256));

  if (!gram_tile) {
    const int64_t c0 = (int64_t)tile * 256 + wave * 64;
    if (c0 >= d) return;
    const int64_t col = c0 + 4 * a;
    f32x4_t acc[4][NB];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[v][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    for (int64_t li = rbeg; li < rend; li += 32) {
      const int64_t rb = (rstart + li) % n;
      uint2 in[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int64_t lr = li + 8 * g + r;
        if (lr < rend) {
          const int64_t row = wrap_row(rb + 8 * g + r, n);
          in[r] = load_row4<FP8>(x + row * ld * ES, col, d);
        } else {
          in[r] = make_uint2(0, 0);
        }
      }
      uint4 bf[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        bf[nb] = *reinterpret_cast<const uint4*>(yb + (((li >> 3) + g) * Kp + nb * 16 + a) * 8);
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
    // lane (j = a, g): acc[v][nb][u] is column c0 + 16g + 4u + v, Y column nb*16 + a
    const int64_t cl = wave * 64 + 16 * g;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      float* dst = pbase + (int64_t)(nb * 16 + a) * 256 + cl;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        store_part(dst + 4 * u,
                   make_float4(acc[0][nb][u], acc[1][nb][u], acc[2][nb][u], acc[3][nb][u]),
                   accumulate);
    }
  } else {
    // Gram tile: A and B fragments are both slices of Y.
    constexpr int MB = (NB + 3) / 4;
    f32x4_t acc[MB][NB];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[m][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    if (wave >= NB) return;
    for (int64_t li = rbeg; li < rend; li += 32) {
      uint4 bf[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        bf[nb] = *reinterpret_cast<const uint4*>(yb + (((li >> 3) + g) * Kp + nb * 16 + a) * 8);
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        const int mb = wave + 4 * m;
        if (mb < NB) {
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(bf[mb]), as_bf16x8(bf[nb]),
                                                                 acc[m][nb], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      const int mb = wave + 4 * m;
      if (mb < NB) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          float* dst = pbase + (int64_t)(nb * 16 + a) * 256 + mb * 16 + 4 * g;
          store_part(dst, make_float4(acc[m][nb][0], acc[m][nb][1], acc[m][nb][2], acc[m][nb][3]),
                     accumulate);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// [Z ; G] partials, float32 data, v_mfma_f32_16x16x4_f32, 16 rows per step.
// ---------------------------------------------------------------------------
template <int NB>
__global__ __launch_bounds__(256) void k_xty_f32(const float* __restrict__ x, int64_t n,
                                                 int64_t d, int64_t ld, int64_t rstart,
                                                 int64_t rows, int64_t rps,
                                                 const float* __restrict__ yb,
                                                 float* __restrict__ part, int ntiles, int nsplit,
                                                 int tile_base, int accumulate) {
  constexpr int Kp = NB * 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int a = lane & 15, g = lane >> 4;
  int tile, split;
  xty_tile_split(ntiles, tile, split);
  tile += tile_base;
  const int64_t rbeg = (int64_t)split * rps;
  const int64_t rend = rbeg + rps < rows ? rbeg + rps : rows;
  float* pbase = part + ((int64_t)(tile - tile_base) * nsplit + split) * Kp * 256;
  const bool gram_tile = (tile == (int)((d + 255) / 256));
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);

  if (!gram_tile) {
    const int64_t c0 = (int64_t)tile * 256 + wave * 64;
    if (c0 >= d) return;
    const int64_t col = c0 + 4 * a;
    f32x4_t acc[4][NB];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[v][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    for (int64_t li = rbeg; li < rend; li += 16) {
      const int64_t rb = (rstart + li) % n;
      float4 in[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int64_t lr = li + 4 * g + s;
        if (lr < rend) {
          const int64_t row = wrap_row(rb + 4 * g + s, n);
          in[s] = load_row4_f32(x + row * ld, col, d);
        } else {
          in[s] = z4;
        }
      }
      float4 bf[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        bf[nb] = *reinterpret_cast<const float4*>(yb + (((li >> 2) + g) * Kp + nb * 16 + a) * 4);
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
    }
    const int64_t cl = wave * 64 + 16 * g;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      float* dst = pbase + (int64_t)(nb * 16 + a) * 256 + cl;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        store_part(dst + 4 * u,
                   make_float4(acc[0][nb][u], acc[1][nb][u], acc[2][nb][u], acc[3][nb][u]),
                   accumulate);
    }
  } else {
    constexpr int MB = (NB + 3) / 4;
    f32x4_t acc[MB][NB];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[m][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    if (wave >= NB) return;
    for (int64_t li = rbeg; li < rend; li += 16) {
      float4 bf[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        bf[nb] = *reinterpret_cast<const float4*>(yb + (((li >> 2) + g) * Kp + nb * 16 + a) * 4);
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        const int mb = wave + 4 * m;
        if (mb < NB) {
          const float am[4] = {bf[mb].x, bf[mb].y, bf[mb].z, bf[mb].w};
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            const float bs[4] = {bf[nb].x, bf[nb].y, bf[nb].z, bf[nb].w};
#pragma unroll
            for (int s = 0; s < 4; ++s)
              acc[m][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(am[s], bs[s], acc[m][nb], 0, 0, 0);
          }
        }
      }
    }
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      const int mb = wave + 4 * m;
      if (mb < NB) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          float* dst = pbase + (int64_t)(nb * 16 + a) * 256 + mb * 16 + 4 * g;
          store_part(dst, make_float4(acc[m][nb][0], acc[m][nb][1], acc[m][nb][2], acc[m][nb][3]),
                     accumulate);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Fixed-order float64 reduction of the partials.
// Z[j][c] = s_j * sum_split part[tile(j)][split][c][j mod 256]   (j < d, c < K)
// G[i][c] = sum_split part[gram][split][c][i]  for i <= c, mirrored.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce_zg(const float* __restrict__ part, int nsplit,
                                                   int Kp, int64_t d, int K,
                                                   const float* __restrict__ scale,
                                                   float* __restrict__ Z, double* __restrict__ G,
                                                   double* __restrict__ Gc, int gram_only,
                                                   int* status) {
  const int64_t gtile = (d + 255) / 256;
  const int64_t nz = gram_only ? 0 : d * K;
  const int64_t ng = (int64_t)K * K;
  const int64_t tile_stride = (int64_t)nsplit * Kp * 256;
  const int64_t gbase = gram_only ? 0 : gtile * tile_stride;
  bool bad = false;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nz + ng;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < nz) {
      // consecutive threads take consecutive rows j for one column c
      const int64_t c = e / d, j = e % d;
      const float* p = part + (j / 256) * tile_stride + c * 256 + (j % 256);
      double s = 0.0;
      for (int t = 0; t < nsplit; ++t) s += (double)p[(int64_t)t * Kp * 256];
      if (scale) s *= (double)scale[j];
      const float zf = (float)s;
      if (!isfinite(zf)) bad = true;
      Z[j * K + c] = zf;
    } else {
      const int64_t f = e - nz;
      const int64_t i = f / K, c = f % K;
      if (i <= c) {
        const float* p = part + gbase + c * 256 + i;
        double s = 0.0;
        for (int t = 0; t < nsplit; ++t) s += (double)p[(int64_t)t * Kp * 256];
        if (!isfinite(s)) bad = true;
        G[i * K + c] = s;
        G[c * K + i] = s;
        if (Gc) {
          Gc[i * K + c] = s;
          Gc[c * K + i] = s;
        }
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

int xty_tiles(int64_t d, int Kp) {
  (void)Kp;
  return (int)((d + 255) / 256) + 1;
}

hipError_t launch_xv(const PassDesc& p, const StreamBufs& b, int64_t i0, int64_t rows,
                     hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  const int64_t rstart = (p.r0 + i0) % p.n;
  const bool small = rows <= 8192;   // short passes (minibatches): 64-row workgroups
  return dispatch_nb(b.Kp, [&](auto nbc) -> hipError_t {
    constexpr int NB = decltype(nbc)::value;
    if (p.dtype == PPCA_F32) {
      if (small) {
        const int64_t grid = cdiv(rows, 64);
        hipLaunchKernelGGL((k_xv_f32<NB, 1>), dim3(grid), dim3(256), 0, s, (const float*)p.x, p.n,
                           p.d, p.ld, rstart, rows, (const float*)b.vop, b.dp, (float*)b.yb);
      } else {
        const int64_t grid = cdiv(rows, 256);
        hipLaunchKernelGGL((k_xv_f32<NB, 4>), dim3(grid), dim3(256), 0, s, (const float*)p.x, p.n,
                           p.d, p.ld, rstart, rows, (const float*)b.vop, b.dp, (float*)b.yb);
      }
    } else {
      const bool fp8 = p.dtype == PPCA_FP8_E4M3;
      const int64_t grid = small ? cdiv(rows, 64) : cdiv(rows, 256);
      auto args = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, s, (const uint8_t*)p.x, p.n, p.d,
                           p.ld, rstart, rows, (const uint16_t*)b.vop, b.dp, (uint16_t*)b.yb);
      };
      if (fp8) {
        if (small) args(k_xv_b16<NB, 1, true>); else args(k_xv_b16<NB, 4, true>);
      } else {
        if (small) args(k_xv_b16<NB, 1, false>); else args(k_xv_b16<NB, 4, false>);
      }
    }
    return hipGetLastError();
  });
}

hipError_t launch_xty(const PassDesc& p, const StreamBufs& b, int64_t i0, int64_t rows,
                      bool accumulate, bool gram_only, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  const int64_t rstart = (p.r0 + i0) % p.n;
  const int ntiles_all = xty_tiles(p.d, b.Kp);
  const int ntiles = gram_only ? 1 : ntiles_all;
  const int tile_base = gram_only ? ntiles_all - 1 : 0;
  const int step = p.dtype == PPCA_F32 ? 16 : 32;
  const int64_t rps = round_up(cdiv(rows, b.nsplit), step);
  const int64_t grid = (int64_t)ntiles * b.nsplit;
  return dispatch_nb(b.Kp, [&](auto nbc) -> hipError_t {
    constexpr int NB = decltype(nbc)::value;
    if (p.dtype == PPCA_F32) {
      hipLaunchKernelGGL((k_xty_f32<NB>), dim3(grid), dim3(256), 0, s, (const float*)p.x, p.n,
                         p.d, p.ld, rstart, rows, rps, (const float*)b.yb, b.part, ntiles,
                         b.nsplit, tile_base, accumulate ? 1 : 0);
    } else if (p.dtype == PPCA_FP8_E4M3) {
      hipLaunchKernelGGL((k_xty_b16<NB, true>), dim3(grid), dim3(256), 0, s, (const uint8_t*)p.x,
                         p.n, p.d, p.ld, rstart, rows, rps, (const uint16_t*)b.yb, b.part, ntiles,
                         b.nsplit, tile_base, accumulate ? 1 : 0);
    } else {
      hipLaunchKernelGGL((k_xty_b16<NB, false>), dim3(grid), dim3(256), 0, s, (const uint8_t*)p.x,
                         p.n, p.d, p.ld, rstart, rows, rps, (const uint16_t*)b.yb, b.part, ntiles,
                         b.nsplit, tile_base, accumulate ? 1 : 0);
    }
    return hipGetLastError();
  });
}

hipError_t launch_reduce_zg(const StreamBufs& b, int64_t d, int K, const float* col_scale,
                            float* Z, double* G, double* G_copy, bool gram_only, int* status,
                            hipStream_t s) {
  const int64_t total = (gram_only ? 0 : d * K) + (int64_t)K * K;
  int64_t grid = cdiv(total, 256);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_reduce_zg, dim3(grid), dim3(256), 0, s, b.part, b.nsplit, b.Kp, d, K,
                     col_scale, Z, G, G_copy, gram_only ? 1 : 0, status);
  return hipGetLastError();
}

}  // namespace ppca
