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

constexpr int kMaxTileBits = 10;   // permute tile: 2^10 complex64 = 8 KiB of LDS
constexpr int kMaxRank = 40;

// out[r][y] = in[r][x], bit p of x moves to bit out_pos[p] of y.
struct PermuteArgs {
  const float2* in;
  float2* out;
  int64_t rows;
  int64_t row_elems;          // 2^rank (both sides)
  int n_tile;                 // bits staged through LDS
  int n_rest;                 // remaining bits (tile index)
  int8_t e_in[kMaxTileBits];  // e-bit j -> input bit position (bits 0.. are input-fastest)
  int8_t f_out[kMaxTileBits]; // f-bit j -> output bit position (bits 0.. are output-fastest)
  int8_t f_to_e[kMaxTileBits];// f-bit j -> e-bit holding the same label
  int8_t r_in[kMaxRank];      // tile-index bit j -> input position
  int8_t r_out[kMaxRank];     // tile-index bit j -> output position
};

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
  int n_m;                    // log2 M
  int nk, nn;                 // log2 K, log2 N (template values)
  int8_t x_kpos[6];           // k bit j -> X bit position
  int8_t x_kins[6];           // X K positions ascending (zero-bit insertion order)
  int8_t s_kpos[6];           // k bit j -> S bit position
  int8_t s_npos[4];           // n bit j -> S bit position
};

// C[r][m][n] = sum_k A[ga(r)][m,k] B[gb(r)][k,n]; A is [M][K] (or [K][M] when trans_a),
// B is [K][N] (or [N][K] when trans_b), C is [M][N].  With k_splits > 1 every split
// writes its partial product to `partial` [split][row][M][N].
struct GemmArgs {
  const float2* A;
  const float2* B;
  float2* C;
  const int32_t* ga;
  const int32_t* gb;
  int64_t rows, a_rows, b_rows;
  int64_t a_row_stride, b_row_stride, c_row_stride;
  int64_t M, N, K;
  int trans_a, trans_b;
  int k_splits;
  int64_t k_chunk;
  float2* partial;
  int config;                 // tile configuration id
};

struct ReduceArgs {           // C[i] = sum_s partial[s][i]
  const float2* partial;
  float2* C;
  int64_t elems;
  int splits;
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

struct SliceLeafArgs {
  const SliceLeafEntry* table;
  const int64_t* prefix;      // [n_entries + 1] element prefix sums
  int n_entries;
  const float2* consts;
  float2* ws;
  const uint64_t* slice_ids;  // device
  int64_t slice_index;
};

// amps[g][mu] (+)= sum over the final tensor's entry for (row_of[g], mu).
struct SliceSumArgs {
  const float2* F;
  double* amps;               // [L][2^n_open] complex128
  const int32_t* row_of;      // [L]
  int64_t L;
  int64_t f_row_stride;
  int n_open;
  int64_t open_stride[64];    // element stride of open qubit t (t = 0 is mu's top bit)
  int overwrite;
};

// Launchers (return hipError_t of the launch).
hipError_t launch_permute(const PermuteArgs& a, hipStream_t s);
hipError_t launch_stream(const StreamArgs& a, hipStream_t s);
hipError_t launch_gemm(const GemmArgs& a, hipStream_t s);
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s);
hipError_t launch_slice_leaves(const SliceLeafArgs& a, int64_t total_elems, hipStream_t s);
hipError_t launch_slice_sum(const SliceSumArgs& a, hipStream_t s);
hipError_t launch_fill_zero(double* p, int64_t n_doubles, hipStream_t s);
// Sum of |amp|^2 over n complex128 values into *out (device double), deterministic.
hipError_t launch_norm(const double* amps, int64_t n, double* partials, int n_partials,
                       double* out, hipStream_t s);
// Inverse-CDF sampler (see tnc.h): writes bitstrings to out[n_samples] (device).
hipError_t launch_sample(const double* amps, int64_t L, int n_open, const uint64_t* closed,
                         const int32_t* open_qubits, int n_qubits, uint64_t seed,
                         int64_t n_samples, double* cum_scratch, uint64_t* out, hipStream_t s);

}  // namespace tnc
