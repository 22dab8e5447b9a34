// Internal declarations shared by the HIP sources of libppca (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/ppca.h"

namespace ppca {

// ---------------------------------------------------------------- constants
constexpr int kMaxK = PPCA_MAX_K;          // largest K = k + l

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------------ device helpers
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

// Report a device-side failure: the first error code written wins.
__device__ inline void set_status(int* status, int code) {
  atomicCAS(status, 0, code);
}

// bf16 bits of the nearest bf16 to a finite float (ties to even).
__device__ inline uint32_t f32_to_bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

__device__ inline float bf16_bits_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

// Exact fp8-e4m3fn -> bf16 bit conversion of one code (every e4m3 value is a
// bf16 value: 3 mantissa bits, exponents 2^-9 .. 2^8).
__device__ inline uint32_t e4m3_to_bf16_bits(uint32_t c) {
  const uint32_t sign = (c & 0x80u) << 8;
  const uint32_t e = (c >> 3) & 0xFu;
  const uint32_t m = c & 0x7u;
  uint32_t mag;
  if (e != 0) {
    mag = ((e + 120u) << 7) | (m << 4);
  } else {
    // subnormal: m * 2^-9, exact in float32
    mag = __float_as_uint((float)m * 0.001953125f) >> 16;
  }
  return sign | mag;
}

// --------------------------------------------------------- host-side launch
// Streaming pass description: rows i = 0 .. nrows-1 of the pass are the data
// rows (r0 + i) mod n.
struct PassDesc {
  const void* x;
  int64_t n, d, ld;
  int32_t dtype;
  const float* col_scale;   // fp8 only
  int64_t r0, nrows;
};

struct StreamBufs {
  const void* vop;      // operand V'^T: [Kp][dp] bf16 (bf16/fp8 data) or f32 (f32 data)
  int64_t dp;           // padded d of the operand
  void* yb;             // Y staging buffer (blocked rows), sized for chunk rows
  int64_t rows_cap;     // rows the staging buffer holds (largest chunk of a pass)
  float* part;          // Z partials [ntiles][nsplit][Kp][xty_cols(Kp)]
  float* gpart;         // G partials [ngpart][Kp][Kp], one per k_xv (or k_ysum) workgroup
  int nsplit;           // row splits of the X^T Y kernel
  int ngpart;           // workgroups of k_xv (fixed for all chunks of a pass)
  int Kp;               // K padded to 16
  int ksplit;           // column splits of a short pass (1 = none)
  float* ypart;         // float32 Y partials [ksplit][rows_cap rounded to 64][Kp]
  bool split = false;   // two-term operand: vop holds hi [Kp][dp] then lo [Kp][dp]
};

// stream kernels (k_stream.hip)
int xv_ksplit(int32_t dtype, int Kp, int64_t d, int64_t rows_cap);   // column splits
int xty_cols(int Kp);              // columns per tile of the X^T Y kernel
int xty_blocks_per_cu(int Kp);     // resident workgroups per CU of the X^T Y kernel
constexpr int kNumCU = 256;        // compute units of an MI355X
int xty_tiles(int64_t d, int Kp);  // column tiles of X in the X^T Y kernel
int xv_grid(int32_t dtype, int Kp, int64_t d, int64_t rows_cap);   // workgroups of k_xv
int xvg_grid(int64_t rows_cap);    // workgroups of the two-term projection pass
hipError_t launch_xv(const PassDesc& p, const StreamBufs& b, int64_t i0, int64_t rows,
                     bool want_y, bool want_g, bool accumulate, hipStream_t s);
// Z (d x K) non-null: written directly by the pass (single row split, single
// chunk); else partials for launch_reduce_zg.
hipError_t launch_xty(const PassDesc& p, const StreamBufs& b, int64_t i0, int64_t rows,
                      bool accumulate, float* Z, int K, int* status, hipStream_t s);
hipError_t launch_reduce_zg(const StreamBufs& b, int64_t d, int K, const float* col_scale,
                            float* Z, double* G, double* G_copy, bool gram_only, int* status,
                            hipStream_t s);

// streaming-read probe (k_probe.hip): workgroups of a mode, and its launch
int probe_grid(int32_t mode);
hipError_t launch_read_probe(const void* x, int64_t n, int64_t row_bytes, int32_t mode,
                             int32_t seg, uint32_t* sink, hipStream_t s);

// single-read power pass (k_fused.hip): bf16 data, Kp a multiple of 32 up to
// 128, d <= 8192; clusters of C = fused_cluster(d) workgroups on one XCD
// (a cooperative launch of 256 workgroups, one per CU)
struct FusedSizes {
  int cluster, nsplit;
  size_t ex_bytes, yb_bytes, flag_bytes, dummy_bytes, part_bytes;
};
struct FusedBufs {
  float* ex;
  uint16_t* yb;
  int* flags;
  float* dummy;
  float* part;   // Z partials [C][nsplit][Kp][256]
};
int fused_cluster(int64_t d);
FusedSizes fused_sizes(int64_t d, int Kp);
bool fused_eligible(int32_t dtype, int64_t d, int Kp);
hipError_t launch_fused_pass(const PassDesc& p, const void* vop, int64_t dp, int Kp,
                             const FusedBufs& fb, int* status, int spin_limit, hipStream_t s);

// dense float64 kernels (k_dense.hip)
// split: bf16 operand as hi = bf16(V) at vop and lo = bf16(V - hi) at
// vop + Kp dp, V_eff = hi + lo (bf16 data only)
hipError_t launch_make_operand(const float* V, int64_t d, int K, int Kp, int64_t dp, int32_t dtype,
                               const float* col_scale, void* vop, bool split, hipStream_t s);
// partial Grams of a (rows x K) matrix A (row stride lda); in_f64 selects the type
int gram_parts(int64_t rows, int K);
hipError_t launch_gram(const void* A, bool in_f64, int64_t rows, int K, int64_t lda,
                       double* parts, double* out, int* status, hipStream_t s);
hipError_t launch_chol_inv(const double* A, int K, double* R, double* Rinv, int* status,
                           hipStream_t s);
hipError_t launch_trmm(const void* A, bool in_f64, int64_t rows, int K, int64_t lda,
                       const double* Rinv, void* out, bool out_f64, int64_t ldo, int* status,
                       hipStream_t s);
// C = alpha * op(A) * B for small K x K / K x k matrices (row-major, float64)
hipError_t launch_small_gemm(const double* A, bool transA, const double* B, double* C, int M,
                             int N, int Kd, int lda, int ldb, int ldc, double alpha,
                             int* status, hipStream_t s);
hipError_t launch_jacobi(const double* H, int K, double* W, double* evals, int max_sweeps,
                         int* status, hipStream_t s);
// Per workgroup and column: the largest |E| entry (its value and row).
struct ColMax {
  float a, v;
  int64_t j;
};
int rotate_blocks(int64_t d, int k);
hipError_t launch_rotate(const float* V, int64_t d, int K, int32_t dtype, bool split,
                         const float* col_scale, const double* M, int k, float* E, ColMax* part,
                         int* flip, int* status, hipStream_t s);
hipError_t launch_operand_gram(const float* V, int64_t d, int K, int32_t dtype, bool split,
                               const float* col_scale, double* parts, double* out, int* status,
                               hipStream_t s);
hipError_t launch_copy_f64(const double* src, double* dst, int64_t count, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

// power method's termination rule and sequential power method (k_seq.hip)
struct SeqState {
  int steps, done;
  double delta;
};
// res[j] (K doubles) = distance of column j of Vn from span(Vo)
hipError_t launch_span_change(const float* Vn, const float* Vo, int64_t d, int K, double* res,
                              hipStream_t s);
hipError_t launch_seq_start(const float* V, int64_t d, int K, int i, float* u, SeqState* st,
                            float* tmp, int* status, hipStream_t s);
hipError_t launch_seq_step(const float* V, int64_t d, int K, int i, const float* Z, float* u,
                           float* w, SeqState* st, double eps, int max_steps, int* status,
                           hipStream_t s);
hipError_t launch_seq_store(float* V, int64_t d, int K, int i, const float* u, hipStream_t s);

// minibatch updates (k_update.hip)
hipError_t launch_sanger_update(float* V, const float* Z, const double* G, int64_t d, int K, int b,
                                double eta, double mu, int nesterov, float* mom, void* vop,
                                int64_t dp, int32_t dtype, const float* col_scale, int* status,
                                hipStream_t s);
int eigengame_blocks(int64_t d, int K);   // blocks of the EigenGame update kernels
size_t eigengame_scratch_doubles(int64_t d, int K);
hipError_t launch_eigengame_update(float* V, const float* Z, const double* G, int64_t d, int K,
                                   int b, double eta, double mu, int nesterov, float* mom,
                                   double* scratch, void* vop, int64_t dp, int32_t dtype,
                                   const float* col_scale, int* status, hipStream_t s);
hipError_t launch_copy_f32(const float* src, float* dst, int64_t count, hipStream_t s);

// data preparation (k_prep.hip)
int prep_row_blocks(int64_t n);
hipError_t launch_center_quantize(const float* x, int64_t n, int64_t d, int64_t ldx,
                                  int32_t out_dtype, void* out, int64_t ldo, float* col_scale,
                                  double* mean_out, double* ws_sums, float* ws_max,
                                  double* ws_mean, hipStream_t s);

// ------------------------------------------------------ grouped problems
// Many independent problems in one call (k_group.hip): bf16 data with
// d <= kGroupMaxD and K <= kGroupMaxK.  A problem belongs to the shape class
// (dci, NB): dci picks the column split of the fused pass (class width dc =
// 64, 128, 256, 512, 768), NB2 = Kp / 32 (K padded to 32).  Its rows are cut into work items;
// the items of all problems are sorted by size and dealt round-robin to the
// persistent workgroups of the fused pass.
constexpr int kGroupMaxD = 768;
constexpr int kGroupMaxK = 64;
constexpr int64_t kGroupMaxLd = 1 << 24;   // 16 rows of X fit a 32-bit byte offset
constexpr int kGroupClasses = 5;
int group_class_width(int dci);          // dc of class dci
int group_row_groups(int dci);           // row groups (waves sharing no rows) of class dci
int group_dci(int64_t d);                // smallest class whose width holds d

struct GProb {
  const uint16_t* x;        // bf16 data [n][ld]
  int64_t n, d, ld;
  int32_t K, Kp, k, cls;    // cls = dci * 2 + NB2 - 1
  int32_t dc, wr;           // class width, row groups of the class
  int32_t nitem, pad;       // number of work items of the problem
  int64_t zbase, gbase;     // float offsets of its item partials: item m of the problem
                            // at zbase + m * wr * Kp * dc and gbase + m * 4 * Kp * Kp
  float* V;                 // [d][K] f32 (caller)
  double* G;                // [K][K] (caller, projection Gram)
  double* B;                // [K][K] (caller)
  float* E;                 // [d][k] (caller, may be null)
  double* evals;            // [k] (caller)
  uint16_t* vop;            // [Kp][dc] bf16 operand hi = bf16(V) (workspace)
  uint16_t* vlo;            // [Kp][dc] bf16 second term lo = bf16(V - hi) (workspace)
  float* Z;                 // [d][K] (workspace)
  double* q1;               // [d][K] (workspace)
  double *A, *R, *Rinv, *H, *W, *ev;   // [K][K], ev [K] (workspace)
};
struct GItem {
  int32_t prob, pad;
  int64_t r0, rows;         // data rows [r0, r0 + rows) of the problem
  int64_t zoff, goff;       // float offsets of the item's Z and G partials
};

hipError_t launch_group_pass(const GProb* probs, const GItem* items, int nitems, int grid,
                             float* zpart, float* gpart, bool want_z, hipStream_t s);
hipError_t launch_group_reduce(const GProb* probs, int nprob, const int* blk0, int nblk,
                               const float* zpart, const float* gpart, bool want_z, int* status,
                               hipStream_t s);
// order: problem indices, largest first (workgroup b takes problem order[b])
// bf16 operand of every problem from its V as it stands (V is not changed)
hipError_t launch_group_operand(const GProb* probs, int nprob, hipStream_t s);
hipError_t launch_group_cholqr2(const GProb* probs, const int* order, int nprob, bool from_v,
                                bool want_b, int* status, hipStream_t s);
hipError_t launch_group_rr(const GProb* probs, const int* order, int nprob, int max_sweeps,
                           int* status, hipStream_t s);

}  // namespace ppca
