// Kernel parameter blocks and launchers (internal to libtnc).
//
// Tensors are complex64, interleaved (float2), laid out [row][dense index] with the
// dense index row-major in the tensor's label order (bit 0 = last label).  Row gathers
// map an output row to an operand row; a null gather means "same row" when the operand
// has as many rows as the output and row 0 otherwise (the operand is broadcast).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tnc {

constexpr int kMaxRank = 40;

// Scale records.  Every tensor carries, per slice copy, a record of kRecWords 32-bit words:
// words 0..kAmaxSlots-1 hold float bits of the largest |re|, |im| of its stored values
// (folded in by atomic maxima from many workgroups; readers take the maximum over the
// slots), word kRecExp the int32 exponent E such that the tensor's true values are the
// stored ones times 2^E.  A kernel contracting A and B multiplies them while loading by
// 2^sA and 2^sB (exact powers of two chosen from their largest components), stores the
// product as it comes out and records E_C = E_A + E_B - sA - sB; the FP64 slice sum
// multiplies by 2^E.  This keeps every stored value inside the floating-point range of the
// arithmetic however small the amplitudes of one slice become.  A null record pointer
// turns the mechanism off for that launch.  Steps are in words per slice copy (0: one
// record shared by every slice).
constexpr int kAmaxSlots = 256;  // atomic-maximum slots per record
constexpr int kRecExp = 256;     // word holding the exponent
constexpr int kRecWords = 264;   // words per record (slots, exponent, padding)

// C[r][m][n] = sum_k X[gx(r)][m (+) k] * S[gs(r)][k, n] for a small S (<= 2^6 x 2^4).
// m enumerates X's free labels in X order; K positions in X are spread anywhere.
struct StreamArgs {
  const float2* X;
  const float2* S;
  float2* C;
  const int32_t* gx;          // nullable
  const int32_t* gs;          // nullable
  int64_t rows;               // output rows
  int64_t x_rows, s_rows;     // operand row counts (for null gathers)
  int64_t x_row_stride, s_row_stride, c_row_stride;
  int64_t nb;                 // slices in this launch
  int64_t x_slice_stride, s_slice_stride, c_slice_stride;   // 0 = shared by every slice
  int n_m;                    // log2 M
  int nk, nn;                 // log2 K, log2 N (template values)
  int8_t x_kpos[6];           // k bit j -> X bit position
  int8_t x_kins[6];           // X K positions ascending (zero-bit insertion order)
  int8_t s_kpos[6];           // k bit j -> S bit position
  int8_t s_npos[4];           // n bit j -> S bit position
  // scale records of X, S and C (see kRecWords)
  const uint32_t* rec_x;
  const uint32_t* rec_s;
  uint32_t* rec_c;
  int64_t rec_x_step, rec_s_step, rec_c_step;
};

// C[r][m][n] = sum_k A[ga(r)][m,k] B[gb(r)][k,n] with C stored [M][N] row-major.
// A and B are read in their own layouts: bit j of the logical index m (k, n) selects bit
// position a_mpos[j] (a_kpos[j] / b_kpos[j], b_npos[j]) of the operand's dense index, so no
// operand is ever permuted.  With fold = 1 the output rows are folded into M:
// m = row * 2^nm + m_local and A's row stride is fold_stride.  With k_splits > 1 every split
// writes its partial product to `partial` [split][row][M][N].
struct GemmArgs {
  const float2* A;
  const float2* B;
  float2* C;
  const int32_t* ga;
  const int32_t* gb;
  int64_t rows, a_rows, b_rows;
  int64_t a_row_stride, b_row_stride, c_row_stride;
  int64_t nb;                 // slices in this launch (partial layout [split][slice][row][M][N])
  int64_t a_slice_stride, b_slice_stride, c_slice_stride;
  int64_t M, N, K;
  int nm, nk, nn;             // log2 of the label groups (M = 2^nm unless folded)
  int fold;
  int64_t fold_stride;
  int a_mfast, b_nfast;       // operand's lowest bit is an m (n) bit: load along m (n)
  int8_t a_mpos[kMaxRank], a_kpos[kMaxRank], b_kpos[kMaxRank], b_npos[kMaxRank];
  int k_splits;
  int64_t k_chunk;
  float2* partial;
  int config;                 // tile configuration id
  int precision;              // 0: complex64 on FP32 MFMA; 1: BF16 hi+lo split in the kernel;
                              // 3: FP16 hi+lo of operands scaled to [2^13, 2^14) per slice
  // Row stacking (stk != nullptr): output rows that share one B row are stacked along M.
  // M is then a multiple of 128 and each output row contributes 2^nm consecutive m; the
  // 128-row block b holds output rows perm[stk[3b]], ..., perm[stk[3b] + stk[3b+1] - 1]
  // and reads B row stk[3b+2].  Such a launch has rows = 1 and k_splits = 1, and A's
  // offsets within one slice fit in 31 bits.
  const int32_t* stk;
  const int32_t* perm;
  int group_m;                // tiles are numbered in groups of group_m tile rows (L2 reuse)
  // scale records of A, B and C (see kRecWords); with k_splits > 1 the reduction folds
  // C's largest component in, the GEMM writes its exponent
  const uint32_t* rec_a;
  const uint32_t* rec_b;
  uint32_t* rec_c;
  int64_t rec_a_step, rec_b_step, rec_c_step;
};

struct ReduceArgs {           // C[i] = sum_s partial[s][i]  (i over every slice of the launch)
  const float2* partial;
  float2* C;
  int64_t elems;
  int splits;
  // optional: C's scale record; the largest |re|, |im| of C per slice (slice = i /
  // slice_elems) is folded into its slots with atomic maxima
  uint32_t* rec;
  int64_t rec_step;
  int64_t slice_elems;
};

// Sliced leaves: for each table entry, out[o] = src[insert(o, slice bits)].
struct SliceLeafEntry {
  int64_t src_off;            // complex64 offset in the constants block
  int64_t dst_off;            // complex64 offset (byte offset / 8) from the workspace base
  int64_t elems_out;          // rows * 2^dense_out
  int32_t dense_out;          // log2 dense elements after slicing
  int32_t n_sl;               // sliced labels held by the leaf
  int8_t pos[8];              // their bit positions in the unsliced dense index, ascending
  int8_t bit[8];              // which bit of the slice id gives each value
};

// Slice s of a launch uses slice id number *base + s (two 64-bit words per id in
// slice_ids) and writes its leaves at dst_off + s * elems_out.
struct SliceLeafArgs {
  const SliceLeafEntry* table;
  const int64_t* prefix;      // [n_entries + 1] element prefix sums
  int n_entries;
  const float2* consts;
  float2* ws;
  const uint64_t* slice_ids;  // device
  const int64_t* base;        // device: index of the launch's first slice in slice_ids
  int64_t nb;
};

// amps[g][mu] (+)= sum over the final tensor's entry for (row_of[g], mu).
// amps is accumulated slice by slice in slice order, whatever the launch's batch size.
struct SliceSumArgs {
  const float2* F;
  double* amps;               // [L][2^n_open] complex128
  const int32_t* row_of;      // [L]
  int64_t L;
  int64_t f_row_stride;
  int64_t nb, f_slice_stride;
  int n_open;
  int64_t open_stride[64];    // element stride of open qubit t (t = 0 is mu's top bit)
  int overwrite;
  const uint32_t* rec_f;      // F's scale record (nullable): values times 2^E
  int64_t rec_f_step;
};

// Launchers (return hipError_t of the launch).
hipError_t launch_stream(const StreamArgs& a, hipStream_t s);
hipError_t launch_gemm(const GemmArgs& a, hipStream_t s);
// whether configuration 5 runs a launch on the narrow-row kernel (k_gemm_rows_narrow),
// which computes in FP32 in every form
bool gemm_rows_narrow_fits(const GemmArgs& a, bool stacked);
// p[0..n) = 0 (clears scale records before their producers fold into them)
hipError_t launch_zero_u32(uint32_t* p, int64_t n, hipStream_t s);
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s);
hipError_t launch_slice_leaves(const SliceLeafArgs& a, int64_t total_elems, hipStream_t s);
hipError_t launch_slice_sum(const SliceSumArgs& a, hipStream_t s);
hipError_t launch_fill_zero(double* p, int64_t n_doubles, hipStream_t s);
// *p = v; *p += v (single-thread kernels: safe inside captured graphs)
hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t s);
hipError_t launch_add_i64(int64_t* p, int64_t v, hipStream_t s);
// Sum of |amp|^2 over n complex128 values into *out (device double), deterministic.
hipError_t launch_norm(const double* amps, int64_t n, double* partials, int n_partials,
                       double* out, hipStream_t s);
// In-group Metropolis chains and frugal rejection sampling (see tnc.h): draws d0 ..
// d0 + n_draws - 1, bitstrings to out[n_draws] (device).  totals: per-group weight sums
// from launch_group_totals.
hipError_t launch_sample_metropolis(const double* amps, int64_t L, int n_open, const uint64_t* closed,
                                    const int32_t* open_qubits, int n_qubits, uint64_t seed,
                                    int64_t d0, int64_t n_draws, int steps, uint64_t* out,
                                    hipStream_t s);
hipError_t launch_group_totals(const double* amps, int64_t L, int n_open, double* totals,
                               hipStream_t s);
hipError_t launch_sample_frugal(const double* amps, const double* totals, int64_t L, int n_open,
                                const uint64_t* closed, const int32_t* open_qubits, int n_qubits,
                                uint64_t seed, int64_t d0, int64_t n_draws, double m, int trials,
                                uint64_t* out, hipStream_t s);
// Inverse-CDF sampler (see tnc.h): writes bitstrings to out[n_samples] (device).
hipError_t launch_sample(const double* amps, int64_t L, int n_open, const uint64_t* closed,
                         const int32_t* open_qubits, int n_qubits, uint64_t seed,
                         int64_t n_samples, double* cum_scratch, uint64_t* out, hipStream_t s);

}  // namespace tnc
