// Device bodies of the one-workgroup dense float64 solvers, shared by the
// single-problem kernels (k_dense.hip) and the grouped kernels (k_group.hip):
//   chol_inv_dev  upper Cholesky factor and its inverse (256 threads, float64
//                 MFMAs for the block products),
//   jacobi_dev    parallel two-sided Jacobi eigensolver (1024 threads, one
//                 16-row block of the eigenvector matrix per workgroup).
// Both use static LDS and report failures through the status word.
#pragma once
#include "ppca_common.h"

namespace ppca {
namespace dev {

constexpr double kEps = 2.220446049250313e-16;

__device__ inline bool status_set(const int* status) {
  return *reinterpret_cast<const volatile int*>(status) != 0;
}

// --------------------------------------------------------------------------
// Upper Cholesky factor R (R^T R = A; written only when R is not null) and
// X = R^-1, K <= KM <= 128, one workgroup of 256 threads, in 16 x 16 blocks
// (the matrix is padded with the identity to a multiple of 16; the padding
// factors to the identity).
//
// Factorisation, for each block row J (two barriers per block row):
//   (1) wavefront 0 factors the diagonal block by row operations on
//       [A_JJ | I]: lane c < 16 holds column c of A_JJ, lane 16 + c column c
//       of the identity, both in registers.  Pivot p scales row p by
//       a_pp^-1/2 (giving row p of R_JJ), then subtracts r_pi times it from
//       every row i > p; the pivot and the r_pi come from other lanes by
//       readlane, so a pivot step has no LDS round trip and no barrier.
//       The identity columns take the same row operations, E A_JJ = R_JJ, so
//       they end as E = R_JJ^-T: lane 16 + c holds row c of X_JJ = R_JJ^-1,
//       written to XD[J].  Pivot test: finite, > K * eps * |a_jj| and > 0,
//       else NOT_SPD;
//   (2) row panel R_J,c = X_JJ^T M_J,c (c > J), one 16 x 16 product per
//       column block on float64 MFMAs;
//   (3) trailing update M_ib,cb -= R_J,ib^T R_J,cb (J < ib <= cb) on MFMAs,
//       with a look-ahead: wavefront 0 updates block (J+1, J+1) first and
//       factors it (step (1) of the next block row) while wavefronts 1-3
//       update the other blocks.
// Inverse, by block columns (one wavefront each, no barrier): for I from
//   the bottom, T_I,cb = sum_{I < kb <= cb} R_I,kb X_kb,cb, then
//   X_I,cb = -X_II T_I,cb, kept transposed in the unused lower blocks of M.
// The panel's column blocks are dealt round-robin to the four wavefronts,
// the other trailing blocks to wavefronts 1-3.  Every sum runs in a fixed
// order.
// --------------------------------------------------------------------------
__device__ inline double bcast_lane(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

typedef double f64x4_t __attribute__((ext_vector_type(4)));

// d += A B for 16 x 16 blocks over k = 0..15 on v_mfma_f64_16x16x4f64: A
// element (i, k) = a(i, k), B element (k, j) = b(k, j).  Lane l supplies
// A[l % 16][4 kc + l / 16] and B[4 kc + l / 16][l % 16]; d[r] is row
// l / 16 + 4 r of column l % 16.
template <typename FA, typename FB>
__device__ inline f64x4_t mma16(f64x4_t d, FA a, FB b) {
  const int l = threadIdx.x & 63, i = l & 15, g = l >> 4;
#pragma unroll
  for (int kc = 0; kc < 4; ++kc)
    d = __builtin_amdgcn_mfma_f64_16x16x4f64(a(i, 4 * kc + g), b(4 * kc + g, i), d, 0, 0, 0);
  return d;
}

// LDS doubles chol_inv_dev<KM> works in (passed in by the caller, so that a
// kernel can reuse the area for its other phases)
template <int KM>
constexpr int chol_lds_doubles() {
  return KM * (KM + 1) + (KM / 16) * 16 * 17 + KM;
}

template <int KM>
__device__ __attribute__((always_inline)) inline void chol_inv_dev(const double* __restrict__ A, int K, double* __restrict__ R,
                                    double* __restrict__ Rinv, int* status, double* lds) {
  constexpr int LDM = KM + 1, BS = 16, NBK = KM / BS, LDX = BS + 1;
  static_assert(KM % BS == 0 && KM <= 128, "block shape");
  double* const M = lds;                     // [KM][LDM]; odd row stride: column reads spread banks
  double* const XD = M + KM * LDM;           // [NBK][BS][LDX]: inverses of the diagonal blocks
  double* const dg = XD + NBK * BS * LDX;    // [KM]
  __shared__ int fail;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, g4 = lane >> 4;
  // one read of the status word for the whole workgroup (another workgroup of
  // a grouped launch may set it meanwhile)
  if (tid == 0) fail = status_set(status) ? 1 : 0;
  __syncthreads();
  if (fail) return;
  __syncthreads();
  const int nbk = (K + BS - 1) / BS, Kp = nbk * BS;
  if (tid == 0) fail = 0;
  // thread -> (column tid % KM, rows tid / KM + RS q): no integer division by
  // K in the loops; batches of 32 loads in flight before the first is used
  constexpr int RS = 256 / KM, LB = 32;
  static_assert(256 % KM == 0, "256 threads");
  const int cc = tid % KM, r0 = tid / KM;
  if (cc < Kp) {
    for (int ib = r0; ib < Kp; ib += LB * RS) {
      double v[LB];
#pragma unroll
      for (int q = 0; q < LB; ++q) {
        const int i = ib + RS * q;
        v[q] = (i < K && cc < K && cc >= i) ? A[i * K + cc] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < LB; ++q) {
        const int i = ib + RS * q;
        if (i >= Kp) break;
        const double w = (i < K && cc < K) ? v[q] : (i == cc ? 1.0 : 0.0);
        M[i * LDM + cc] = w;
        if (i == cc) dg[i] = w;
      }
    }
  }
  __syncthreads();
  // (1) diagonal block J and its inverse, wavefront 0 only (lanes >= 32
  // repeat lanes 0..31 and store nothing)
  auto factor_diag = [&](int J) {
    const int j0 = J * BS, c = l16;
    const bool ip = (lane & 16) != 0;            // identity column
    double col[BS], tol[BS];
#pragma unroll
    for (int i = 0; i < BS; ++i) {
      col[i] = ip ? (i == c ? 1.0 : 0.0) : ((i <= c) ? M[(j0 + i) * LDM + j0 + c] : 0.0);
      tol[i] = (double)K * kEps * fabs(dg[j0 + i]);
    }
    bool ok = true;
#pragma unroll
    for (int p = 0; p < BS; ++p) {
      const double piv = bcast_lane(col[p], p);
      // uniform: every lane holds the same pivot; after a failure the values
      // are garbage and are not stored (no short-circuit: no branch in the
      // pivot chain)
      ok = ok & (bool)isfinite(piv) & (piv > tol[p]) & (piv > 0.0);
      const double rinv = rsqrt(fabs(piv));
      // row p scaled: r_pc in block lane c >= p (r_pp = |a_pp| rinv), zero
      // left of the diagonal; e_pc in identity lane c
      const double sp = ip ? col[p] * rinv
                           : ((c == p) ? fabs(piv) * rinv : ((c > p) ? col[p] * rinv : 0.0));
#pragma unroll
      for (int i = p + 1; i < BS; ++i) {
        const double rpi = bcast_lane(sp, i);    // r_pi, from block lane i
        if (ip || i <= c) col[i] = fma(-rpi, sp, col[i]);
      }
      col[p] = sp;
    }
    if (!ok) {
      if (lane == 0) fail = 1;
    } else if (lane < BS) {
#pragma unroll
      for (int i = 0; i < BS; ++i)
        if (i <= c) M[(j0 + i) * LDM + j0 + c] = col[i];
    } else if (lane < 2 * BS) {
      // row c of X_JJ (zero left of the diagonal)
#pragma unroll
      for (int i = 0; i < BS; ++i) XD[J * BS * LDX + c * LDX + i] = (i >= c) ? col[i] : 0.0;
    }
  };
  // (3) M_ib,cb -= R_J,ib^T R_J,cb for one upper block (lower half of a
  // diagonal block untouched)
  auto trail_block = [&](int j0, int ib, int cb) {
    f64x4_t d;
#pragma unroll
    for (int r = 0; r < 4; ++r) d[r] = M[(ib * BS + g4 + 4 * r) * LDM + cb * BS + l16];
    d = mma16(d, [&](int i, int k) { return -M[(j0 + k) * LDM + ib * BS + i]; },
              [&](int k, int j) { return M[(j0 + k) * LDM + cb * BS + j]; });
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (ib != cb || g4 + 4 * r <= l16) M[(ib * BS + g4 + 4 * r) * LDM + cb * BS + l16] = d[r];
  };
  if (wave == 0) factor_diag(0);
  __syncthreads();
  if (fail) {
    if (tid == 0) set_status(status, PPCA_ERR_NOT_SPD);
    return;
  }
  for (int J = 0; J + 1 < nbk; ++J) {
    const int j0 = J * BS;
    // (2) row panel R_J,cb = X_JJ^T M_J,cb
    const double* xj = XD + J * BS * LDX;
    for (int cb = J + 1 + wave; cb < nbk; cb += 4) {
      f64x4_t d = f64x4_t{0.0, 0.0, 0.0, 0.0};
      d = mma16(d, [&](int i, int k) { return xj[k * LDX + i]; },
                [&](int k, int j) { return M[(j0 + k) * LDM + cb * BS + j]; });
#pragma unroll
      for (int r = 0; r < 4; ++r) M[(j0 + g4 + 4 * r) * LDM + cb * BS + l16] = d[r];
    }
    __syncthreads();
    // (3) trailing update of the upper blocks (ib, cb), J < ib <= cb, with a
    // look-ahead: wavefront 0 updates the next diagonal block and factors it
    // (1) while the other three update the rest
    const int nt = nbk - 1 - J;
    if (wave == 0) {
      trail_block(j0, J + 1, J + 1);
      __builtin_amdgcn_wave_barrier();   // same wavefront: LDS order is program order
      factor_diag(J + 1);
    } else {
      for (int q = wave; q < nt * (nt + 1) / 2; q += 3) {   // q = 0 is block (J+1, J+1)
        int ib = 0, rem = q;
        while (rem >= nt - ib) {
          rem -= nt - ib;
          ++ib;
        }
        trail_block(j0, J + 1 + ib, J + 1 + ib + rem);
      }
    }
    __syncthreads();
    if (fail) {
      if (tid == 0) set_status(status, PPCA_ERR_NOT_SPD);
      return;
    }
  }
  // Inverse, one block column at a time with no barrier: wavefront w takes
  // columns nbk-1-w and w (the work of column cb grows like cb^2).  For
  // I = cb-1 .. 0: T = sum_{I < kb <= cb} R_I,kb X_kb,cb, X_I,cb = -X_II T
  // (T stays in the accumulators: their layout is the B operand's).  X_I,cb
  // goes transposed into the unused lower block (cb, I) of M, so R stays
  // whole for the other columns.
  auto inv_column = [&](int cb) {
    for (int I = cb - 1; I >= 0; --I) {
      const int i0 = I * BS;
      f64x4_t t = f64x4_t{0.0, 0.0, 0.0, 0.0};
      for (int kb = I + 1; kb <= cb; ++kb) {
        if (kb == cb)
          t = mma16(t, [&](int i, int k) { return M[(i0 + i) * LDM + kb * BS + k]; },
                    [&](int k, int j) { return XD[cb * BS * LDX + k * LDX + j]; });
        else
          t = mma16(t, [&](int i, int k) { return M[(i0 + i) * LDM + kb * BS + k]; },
                    [&](int k, int j) { return M[(cb * BS + j) * LDM + kb * BS + k]; });
      }
      // B operand element (4 kc + g4, l16) of the product is t[kc]
      f64x4_t x = f64x4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kc = 0; kc < 4; ++kc)
        x = __builtin_amdgcn_mfma_f64_16x16x4f64(-XD[I * BS * LDX + l16 * LDX + 4 * kc + g4],
                                                 t[kc], x, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) M[(cb * BS + l16) * LDM + i0 + g4 + 4 * r] = x[r];
    }
  };
  if (nbk - 1 - wave >= wave) {
    inv_column(nbk - 1 - wave);
    if (wave < nbk - 1 - wave) inv_column(wave);
  }
  __syncthreads();
  // R (upper blocks of M) and R^-1 (diagonal blocks in XD, the others
  // transposed in the lower blocks of M) out
  if (cc < K) {
#pragma unroll 4
    for (int i = r0; i < K; i += RS) {
      const int ib = i / BS, cb = cc / BS;
      if (R) R[i * K + cc] = cc >= i ? M[i * LDM + cc] : 0.0;
      Rinv[i * K + cc] = ib < cb    ? M[cc * LDM + i]
                         : ib > cb  ? 0.0
                         : cc >= i ? XD[ib * BS * LDX + (i % BS) * LDX + cc % BS]
                                    : 0.0;
    }
  }
}

// --------------------------------------------------------------------------
// Parallel two-sided Jacobi (round-robin pairing), float64, K <= 128.
// Every workgroup runs the identical iteration on its own copy of A (in LDS)
// and accumulates the 16 rows [16*blockIdx.x, 16*blockIdx.x + 16) of the
// eigenvector matrix W.  Each round rotates K/2 disjoint pairs at once:
// A <- J^T A J, W <- W J, with the classical rotation that zeroes a_pq
// (tau = (a_qq - a_pp)/(2 a_pq), t = sign(tau)/(|tau| + sqrt(1+tau^2))).
// A rotation round updates the upper triangle of A only (one 2x2 block of
// the pair-by-pair partition per thread, four reads and four writes).
// Stops when off(A) <= 1e-15 ||A||_F or a sweep rotates nothing.
// Output: evals[K] descending; Ws[i][rank] = W[i][col] sorted to match.
constexpr int kJacRows = 16;

__device__ inline int rr_pos(int m, int r, int kpad) {
  return m == 0 ? 0 : 1 + (m - 1 + r) % (kpad - 1);
}

__device__ double block_sum(double v, double* red) {
  // 1024 threads -> 16 waves
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
  __syncthreads();
  return t;
}

template <int KM, int JR = kJacRows>
__device__ inline void jacobi_dev(const double* __restrict__ H, int K, double* __restrict__ Ws,
                                  double* __restrict__ evals, int max_sweeps, int* status,
                                  int rowblk) {
  __shared__ double A[KM * (KM + 1)];   // row stride kpad + 1: column accesses spread banks
  __shared__ double Wl[JR * KM];
  __shared__ double2 rot[KM / 2];      // (c, s) of pair i
  __shared__ int2 pq[KM / 2];          // (p, q) of pair i, p < q
  __shared__ double red[16];
  __shared__ int any_rot;
  __shared__ int rank_of[KM];
  const int tid = threadIdx.x;
  // one read of the status word for the whole workgroup
  if (tid == 0) any_rot = status_set(status) ? 1 : 0;
  __syncthreads();
  if (any_rot) return;
  __syncthreads();
  const int kpad = K + (K & 1);     // index K is a dummy when K is odd
  const int npair = kpad / 2;
  const int la = kpad + 1;          // LDS row stride of A
  const int row0 = rowblk * JR;
  // rotations update the upper triangle only: element (i, j) lives at
  // (min, max) (the load writes both triangles; the lower one goes stale)
  auto up = [la](int i, int j) { return i < j ? i * la + j : j * la + i; };
  // H in batches of 8 elements per thread (all loads in flight before use)
  for (int e0 = tid; e0 < kpad * kpad; e0 += 8 * 1024) {
    double hv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + 1024 * u;
      const int i = e / kpad, j = e % kpad;
      hv[u] = (e < kpad * kpad && i < K && j < K) ? 0.5 * (H[i * K + j] + H[j * K + i]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + 1024 * u;
      if (e < kpad * kpad) A[(e / kpad) * la + (e % kpad)] = hv[u];
    }
  }
  for (int e = tid; e < JR * kpad; e += blockDim.x) {
    const int r = e / kpad, j = e % kpad;
    Wl[e] = (row0 + r == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  double loc = 0.0;
  for (int e = tid; e < kpad * kpad; e += blockDim.x) {
    const int i = e / kpad, j = e % kpad;
    loc += A[i * la + j] * A[i * la + j];
  }
  const double fro = sqrt(block_sum(loc, red));
  bool converged = (K <= 1) || fro == 0.0;
  for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
    loc = 0.0;
    for (int e = tid; e < kpad * kpad; e += blockDim.x) {
      const int i = e / kpad, j = e % kpad;
      if (i != j) loc += A[up(i, j)] * A[up(i, j)];
    }
    const double off = sqrt(block_sum(loc, red));
    if (off <= 1e-15 * fro) {
      converged = true;
      break;
    }
    if (tid == 0) any_rot = 0;
    __syncthreads();
    for (int r = 0; r < kpad - 1; ++r) {
      if (tid < npair) {
        int p = rr_pos(tid, r, kpad), q = rr_pos(kpad - 1 - tid, r, kpad);
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < K) {
          const double apq = A[p * la + q], app = A[p * la + p], aqq = A[q * la + q];
          if (!(fabs(apq) <= 1e-300 || fabs(apq) < 0.1 * kEps * sqrt(fabs(app * aqq)))) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + hypot(1.0, tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            any_rot = 1;
          }
        }
        pq[tid] = make_int2(p, q);
        rot[tid] = make_double2(c, s);
      }
      __syncthreads();
      // 2x2 blocks (bi <= bj), each updated by one thread in the upper
      // triangle; thread t takes bi = t/16 + 64m, bj = t%16 + 16m' (no division)
      for (int bi = tid >> 4; bi < npair; bi += 64) {
        const int2 pqi = pq[bi];
        const double2 ri = rot[bi];
        const int pi = pqi.x, qi = pqi.y;
        const double ci = ri.x, si = ri.y;
        for (int bj = tid & 15; bj < npair; bj += 16) {
          if (bi > bj) continue;
          const int2 pqj = pq[bj];
          const double2 rj = rot[bj];
          const int pj = pqj.x, qj = pqj.y;
          const double cj = rj.x, sj = rj.y;
          if (si == 0.0 && sj == 0.0) continue;
          const int ia = up(pi, pj), ib = up(pi, qj), ie = up(qi, pj), iff = up(qi, qj);
          const double a = A[ia], b = A[ib];
          const double e0 = A[ie], f = A[iff];
          const double a1 = ci * a - si * e0, b1 = ci * b - si * f;
          const double e1 = si * a + ci * e0, f1 = si * b + ci * f;
          double a2 = cj * a1 - sj * b1, b2 = sj * a1 + cj * b1;
          double e2 = cj * e1 - sj * f1, f2 = sj * e1 + cj * f1;
          if (bi == bj) {
            A[ia] = a2;
            A[iff] = f2;
            A[ib] = 0.0;
          } else {
            A[ia] = a2;
            A[ib] = b2;
            A[ie] = e2;
            A[iff] = f2;
          }
        }
      }
      // W rows of this workgroup: thread t takes row t/64 and pair t%64
      for (int lr = tid >> 6; lr < JR; lr += 16) {
        for (int i = tid & 63; i < npair; i += 64) {
          const double2 r = rot[i];
          const double s = r.y;
          if (s == 0.0) continue;
          const double c = r.x;
          const int p = pq[i].x, q = pq[i].y;
          const double wp = Wl[lr * kpad + p], wq = Wl[lr * kpad + q];
          Wl[lr * kpad + p] = c * wp - s * wq;
          Wl[lr * kpad + q] = s * wp + c * wq;
        }
      }
      __syncthreads();
    }
    if (!any_rot) converged = true;
    __syncthreads();
  }
  if (!converged) {
    loc = 0.0;
    for (int e = tid; e < kpad * kpad; e += blockDim.x) {
      const int i = e / kpad, j = e % kpad;
      if (i != j) loc += A[up(i, j)] * A[up(i, j)];
    }
    const double off = sqrt(block_sum(loc, red));
    if (off > 1e-15 * fro) {
      if (tid == 0) set_status(status, PPCA_ERR_NO_CONVERGENCE);
      return;
    }
  }
  // stable descending ranks
  for (int i = tid; i < K; i += blockDim.x) {
    const double ti = A[i * la + i];
    int rk = 0;
    for (int j = 0; j < K; ++j) {
      const double tj = A[j * la + j];
      rk += (tj > ti) || (tj == ti && j < i);
    }
    rank_of[i] = rk;
    if (rowblk == 0) evals[rk] = ti;
  }
  __syncthreads();
  for (int e = tid; e < JR * K; e += blockDim.x) {
    const int lr = e / K, i = e % K;
    if (row0 + lr < K) Ws[(row0 + lr) * K + rank_of[i]] = Wl[lr * kpad + i];
  }
}

}  // namespace dev
}  // namespace ppca
