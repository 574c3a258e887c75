// Host-side launchers shared between the translation units of the library.
#pragma once

#include "common.hpp"

namespace lk {

// ---- embeddings and the fused kernel product (kmv.hip) ----

// Bytes of a prepared embedding copy of `rows` rows in precision `prec`.
size_t embed_bytes(int64_t rows, int dp, int prec);

// Writes the prepared copy of E (rows x d, float64) padded to dp columns:
//   F64:  sqrt(s) * e                      (kernel uses exp)
//   F32:  fp32(sqrt(s log2 e) * e)         (kernel uses exp2)
//   BF16: bf16(fp32(sqrt(s log2 e) * e))   (kernel uses exp2)
hipError_t prep_embed(const double* E, int64_t rows, int d, int dp, double scale, int prec,
                      void* out, hipStream_t st);

constexpr int kMaxSplit = 64;   // largest number of column ranges of one product

// Schedule of the symmetric square product  (bfloat16 / float32, dp <= 64).
// G = exp2(s E E^T) is symmetric, so each off-diagonal entry is formed once
// and used twice: row blocks of kSymRows rows meet column stages of kSymCols
// key rows only on or right of the block diagonal (T stages in all); the
// stages right of the diagonal also add their transposed products into the
// stage's columns.  The stage list runs through the row blocks in the order
// 0, nrb - 1, 1, nrb - 2, ... (a long row block, then a short one), each
// block's stages in column order; a fixed grid of kSymGrid blocks takes equal
// contiguous runs of it, so that every block does the same work and meets few
// row blocks.
// Partials: `rs` row slots per row block (one per block whose run meets it),
// then one column slot per row block:
//   part[k n + i]          k < slots(block of i):   row sums of i
//   part[(rs + I) n + i]   I < row block of i:       transposed sums of i
// With f32 (the bfloat16 kernel) the slots are float32, same positions in
// (float*)part: each is a float64 sum rounded once, far inside the bfloat16
// product's accuracy, and the partials' traffic halves.
constexpr int kSymRows = 256;
constexpr int kSymCols = 128;
constexpr int kSymGrid = 256;
constexpr int kSymMaxRowBlocks = 512;
struct SymPlan {
  int nrb;      // row blocks
  int ncs;      // column stages
  int grid;     // blocks of the launch
  int rs;       // row slots (largest count over the row blocks)
  int f32;      // slots stored as float32
  int64_t T;    // stages
};
// row block at position t of the order, and the position of row block I
__host__ __device__ inline int64_t sym_rowblock_at(int64_t t, int64_t nrb) { return (t & 1) ? nrb - 1 - (t >> 1) : (t >> 1); }
__host__ __device__ inline int64_t sym_pos_of(int64_t I, int64_t nrb) { return 2 * I <= nrb - 1 ? 2 * I : 2 * (nrb - 1 - I) + 1; }
// first stage of the row block at position t (row block I has ncs - 2 I stages;
// the pair at positions 2k, 2k + 1 has 2 ncs - 2 nrb + 2)
__host__ __device__ inline int64_t sym_pos_start(int64_t t, int64_t nrb, int64_t ncs) {
  const int64_t k = t >> 1;
  const int64_t P = 2 * ncs - 2 * nrb + 2;
  return (t & 1) ? k * P + (ncs - 2 * k) : k * P;
}
// block whose run [T b / G, T (b + 1) / G) holds stage s
__host__ __device__ inline int64_t sym_block_of(int64_t s, int64_t G, int64_t T) { return ((s + 1) * G - 1) / T; }

// Row blocks x column ranges of one product (sym: the symmetric schedule).
struct KmvPlan {
  int nsplit;
  int64_t cols_per_split;
  int rowblocks;
  int sym;
  SymPlan sp;
};
KmvPlan kmv_plan(int64_t m, int64_t n, int prec);
// plan of the square product of n rows with itself (symmetric when it applies)
KmvPlan kmv_plan_square(int64_t n, int dp, int prec);
int kmv_rows_per_block(int prec);
// doubles of the partial buffer the products of an (m x n) problem may use
size_t kmv_part_elems(int64_t m, int64_t n);

// Layout of the partial sums of one product, and their fixed-order sum.  The
// readers take the slot type once per call (float32 slots: sp.f32) and then
// issue their loads in batches, as for float64 slots.
struct PartSum {
  int nsplit;
  int sym;
  SymPlan sp;
  // s += part[(first + k) m + i] for k < count, in order; the loads are
  // issued eight at a time so that their latencies overlap
  template <typename PT>
  __device__ __forceinline__ static void add_run(double& s, const PT* __restrict__ part, int64_t m, int64_t i,
                                                 int64_t first, int64_t count) {
    int64_t k = 0;
    for (; k + 8 <= count; k += 8) {
      PT v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = part[(first + k + q) * m + i];
#pragma unroll
      for (int q = 0; q < 8; ++q) s += (double)v[q];
    }
    for (; k < count; ++k) s += (double)part[(first + k) * m + i];
  }
  // row slots of row i (count nr) and the offset of its column slots
  __device__ __forceinline__ void row_list(int64_t i, int64_t& nr, int64_t& cnt, int64_t& c0) const {
    nr = nsplit;
    cnt = nsplit;
    c0 = 0;
    if (sym) {
      const int64_t I = i / kSymRows;
      const int64_t t = sym_pos_of(I, sp.nrb);
      const int64_t b0 = sym_block_of(sym_pos_start(t, sp.nrb, sp.ncs), sp.grid, sp.T);
      const int64_t b1 = sym_block_of(sym_pos_start(t + 1, sp.nrb, sp.ncs) - 1, sp.grid, sp.T);
      nr = b1 - b0 + 1;
      cnt = nr + I;
      c0 = sp.rs - nr;
    }
  }
  template <typename PT>
  __device__ __forceinline__ double row_t(const PT* __restrict__ part, int64_t m, int64_t i) const {
    double s = 0.0;
    int64_t nr, cnt, c0;
    row_list(i, nr, cnt, c0);
    add_run(s, part, m, i, 0, nr);
    if (cnt > nr) add_run(s, part, m, i, sp.rs, cnt - nr);
    return s;
  }
  __device__ __forceinline__ double row(const double* __restrict__ part, int64_t m, int64_t i) const {
    return sym && sp.f32 ? row_t(reinterpret_cast<const float*>(part), m, i) : row_t(part, m, i);
  }
  // the same list of partials of row i (row slots, then column slots), but
  // only positions q, q + Q, q + 2 Q, ... of it, added in that order
  template <typename PT>
  __device__ __forceinline__ double row_strided_t(const PT* __restrict__ part, int64_t m, int64_t i, int q,
                                                  int Q) const {
    int64_t nr, cnt, c0;
    row_list(i, nr, cnt, c0);
    double s = 0.0;
    int64_t k = q;
    for (; k + 7 * Q < cnt; k += 8 * Q) {
      PT v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t kk = k + u * Q;
        v[u] = part[(kk < nr ? kk : c0 + kk) * m + i];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) s += (double)v[u];
    }
    for (; k < cnt; k += Q) s += (double)part[(k < nr ? k : c0 + k) * m + i];
    return s;
  }
  __device__ __forceinline__ double row_strided(const double* __restrict__ part, int64_t m, int64_t i, int q,
                                                int Q) const {
    return sym && sp.f32 ? row_strided_t(reinterpret_cast<const float*>(part), m, i, q, Q)
                         : row_strided_t(part, m, i, q, Q);
  }
  // row_strided with all (at most MAXC) of the thread's loads issued at once;
  // the same sum, in the same order; longer lists take row_strided
  template <int MAXC, typename PT>
  __device__ __forceinline__ double row_strided_all_t(const PT* __restrict__ part, int64_t m, int64_t i, int q,
                                                      int Q) const {
    int64_t nr, cnt, c0;
    row_list(i, nr, cnt, c0);
    if (cnt > q + (int64_t)MAXC * Q) return row_strided_t(part, m, i, q, Q);
    PT v[MAXC];
#pragma unroll
    for (int u = 0; u < MAXC; ++u) {
      const int64_t kk = q + (int64_t)u * Q;
      v[u] = kk < cnt ? part[(kk < nr ? kk : c0 + kk) * m + i] : (PT)0;
    }
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < MAXC; ++u)
      if (q + (int64_t)u * Q < cnt) s += (double)v[u];
    return s;
  }
  template <int MAXC>
  __device__ __forceinline__ double row_strided_all(const double* __restrict__ part, int64_t m, int64_t i, int q,
                                                    int Q) const {
    return sym && sp.f32 ? row_strided_all_t<MAXC>(reinterpret_cast<const float*>(part), m, i, q, Q)
                         : row_strided_all_t<MAXC>(part, m, i, q, Q);
  }
};
inline PartSum part_sum(const KmvPlan& pl) {
  PartSum ps;
  ps.nsplit = pl.nsplit;
  ps.sym = pl.sym;
  ps.sp = pl.sp;
  return ps;
}

// One fused product  out_i = lam * pself_i + sum_j exp(<q_i, k_j>) p_j  (exp2 for
// the float32 / bfloat16 prepared copies).  All vectors are float64.  The
// float64 kernel accumulates in float64; the float32 / bfloat16 kernels sum the
// products of one LDS stage (4 per lane and row) in float32 and add each stage
// sum into a float64 accumulator, so the rounding of the sums does not grow
// with n.
struct KmvArgs {
  const void* Q;        // prepared query rows (m x dp)
  int64_t m;
  const void* K;        // prepared key rows (n x dp)
  int64_t n;
  const double* p;      // vector over the key rows
  double* part;         // nsplit x m column-range partials
  int64_t cps;          // filled by kmv_run
  int nsplit;           // filled by kmv_run
  int mode;             // 0: partials only; 1: finished output
  double lam;           // lambda (0 for the rectangular product)
  const double* pself;  // vector over the output rows for lam * pself; null: none
  double* out;          // output vector (mode 1)
  PcgScalars* S;        // when set, the launch is skipped once S->done
  int pcg_step;         // 1: this product starts a PCG iteration (advances S->kcur)
  PartSum ps;           // filled by kmv_run
  // symmetric schedule only (null: not formed): one float64 partial per block
  // of  p^T (lam I + G) p  = sum_i p_i (lam p_i + partials of row i), the
  // curvature of a CG step, taken from the partial sums as they are written
  double* pap;
  // symmetric schedule inside PCG with a low-rank preconditioner (null: p is
  // used as given): the kernel uses the conjugated direction theta + beta p,
  // formed on the fly with beta = (sum of the grz <= 1024 partials rzp of
  // r^T theta) / S->rzold (0 while S->first); block 0 records beta and the
  // new r^T theta in S.  p itself is left unchanged (the step update stores
  // the new direction after this launch).
  const double* theta;
  const double* rzp;
  int grz;
  // stored kernel matrix of this product's precision (float64 or float32
  // tiles of the symmetric schedule, see kmat_build); null: recomputed
  const void* kmat;
};
hipError_t kmv_run(int prec, int dp, const KmvPlan& pl, KmvArgs A, hipStream_t st);

// Stored kernel matrix for square products that take the symmetric schedule
// (kmat_applies): the schedule's stage tiles, 256 x 128 row-major each, in
// stage order, entries exp(s <e_i, e_j>) computed as the float64 kernel does
// and stored as float64 (prec F64) or rounded to float32 (prec F32); entries
// outside n x n are zero.  kmat_bytes: its size; kmat_build: fill it from the
// float64 prepared embeddings e64 (dp columns).
bool kmat_applies(int64_t n, int dp);
size_t kmat_bytes(int64_t n, int prec);
hipError_t kmat_build(int dp, const double* e64, int64_t n, int prec, void* out, hipStream_t st);

// Products of several problems in one launch: block b computes tile
// (problem, row block, column range) = tiles_dev[3 b .. 3 b + 2] with the
// problem's arguments As_dev[problem] (cps and nsplit filled in).  With
// `finish`, a second launch writes out = lam pself + the partials for every
// problem whose mode is 1 (max_m: the largest row count).
hipError_t kmv_run_batch(int prec, int dp, int count, const KmvArgs* As_dev, const int* tiles_dev, int ntiles,
                         bool finish, int64_t max_m, hipStream_t st);
// Symmetric bfloat16 products (mode 0) of several maps in one launch: maps
// list_dev[0 .. count) with arguments As_dev[map] and square plans Ps_dev[map]
// (kmv_plan_square(n, dp, LAKER_BF16).sp, symmetric); kmv_sym16(dp, prec): the
// precisions and widths whose symmetric products this launch covers.
bool kmv_sym16(int dp, int prec);
hipError_t kmv_run_sym16_batch(int dp, int count, const KmvArgs* As_dev, const SymPlan* Ps_dev,
                               const int* list_dev, hipStream_t st);

// ---- multi right-hand-side product and the fit (fit.hip) ----

}  // namespace lk
