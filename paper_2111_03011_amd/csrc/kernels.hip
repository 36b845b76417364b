// HIP kernels of the contraction path, written for CDNA4 (gfx950, wave64).
//
//   k_stream       big tensor x small tensor, reading the big one in its own layout
//                  (the small operand's labels may sit at any bit positions)
//   k_gemm         complex64 GEMM on the FP32 matrix cores: the interleaved complex A is
//                  used as a real M x 2K matrix and B is expanded on the fly into the
//                  2K x 2N real embedding [[Br, Bi], [-Bi, Br]], so one
//                  v_mfma_f32_32x32x2f32 consumes exactly one complex k; both operands
//                  are read in their stored label order (per-slot scattered offsets), so
//                  the path needs no transposes
//   k_reduce(_wide) split-K partial sums, fixed order
//   k_slice_leaves per-slice instantiation of the leaves that hold sliced bonds
//   k_slice_sum    FP64 accumulation of a slice's result into psi_hat
//   k_norm_*       FP64 sum of |amp|^2, two fixed-order passes
//   k_sample_*     inverse-CDF sampling with SplitMix64 uniforms
#include "tnc_kernels.h"

#include <cstdlib>

namespace tnc {

namespace {

constexpr int kThreads = 256;

// Fold per-lane maxima m >= 0 into the kAmaxSlots slots of record copy `slice`,
// amax[slice * step + j], with atomic maxima on the float bits (non-negative floats order
// like their bits); the slot is a hash of the workgroup index, which spreads the atomics of
// a large output over many addresses, and readers take the maximum over the slots
// (amax_read).  Every lane of the wave calls this; a lane without an element passes
// slice = -1.  When the lanes with an element share one slice the wave reduces first and
// issues one atomic.
__device__ __forceinline__ void amax_commit(float m, int64_t slice, uint32_t* amax, int64_t step) {
  amax += (blockIdx.x + 7u * blockIdx.y + 13u * blockIdx.z) & (kAmaxSlots - 1);
  int64_t s0 = slice;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int64_t o = __shfl_xor(s0, off);
    s0 = s0 > o ? s0 : o;
  }
  if (s0 < 0) return;
  if (__all(slice == s0 || slice < 0)) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0 && m > 0.f) atomicMax(amax + s0 * step, __float_as_uint(m));
  } else if (slice >= 0 && m > 0.f) {
    atomicMax(amax + slice * step, __float_as_uint(m));
  }
}

// maximum over a record's kAmaxSlots slots (lane j reads slots j, j + 64, ...; every lane
// of the wave gets the result)
__device__ __forceinline__ uint32_t amax_read(const uint32_t* slots) {
  const int lane = threadIdx.x & 63;
  uint32_t v = 0;
#pragma unroll
  for (int k = 0; k < kAmaxSlots / 64; ++k) {
    const uint32_t o = slots[lane + 64 * k];
    v = v > o ? v : o;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t o = __shfl_xor(v, off);
    v = v > o ? v : o;
  }
  return v;
}

// amax_commit for a workgroup whose lanes all hold elements of one slice: the four waves'
// maxima meet in LDS and one atomic maximum goes out per workgroup.  Every thread of the
// workgroup calls it (it synchronises the workgroup).
__device__ __forceinline__ void amax_commit_wg(float m, int64_t slice, uint32_t* amax, int64_t step) {
  __shared__ float red[16];   // up to 16 waves per workgroup
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    float w = red[0];
    for (int i = 1; i < int(blockDim.x >> 6); ++i) w = fmaxf(w, red[i]);
    if (w > 0.f)
      atomicMax(amax + slice * step + ((blockIdx.x + 7u * blockIdx.y + 13u * blockIdx.z) & (kAmaxSlots - 1)),
                __float_as_uint(w));
  }
}

// Scale shift of an operand from its largest component (float bits): the FP32 forms
// (f16 = false) leave operands whose largest component lies in [2^-20, 2^21) alone and
// bring the others to [1, 2); the FP16 form brings it to [2^13, 2^14) (exponents clamped
// to [-110, 127]).  An all-zero operand is not scaled.  The result lies in [-126, 127].
__device__ __forceinline__ int rec_shift(uint32_t amax_bits, bool f16) {
  const int e = int((amax_bits >> 23) & 0xffu) - 127;   // -127 for zero and subnormals
  if (f16) return 13 - (e < -110 ? -110 : e);
  if (amax_bits == 0u || (e >= -20 && e <= 20)) return 0;
  return e > 126 ? -126 : -e;
}

// 2^k for k in [-126, 127]
__device__ __forceinline__ float pow2f(int k) { return __uint_as_float(uint32_t(127 + k) << 23); }

// Shift and exponent of record copy `slice` (every lane of the wave calls it).
__device__ __forceinline__ void rec_load(const uint32_t* rec, int64_t step, int64_t slice, bool f16,
                                         int& shift, int& expo) {
  const uint32_t* r = rec + slice * step;
  shift = rec_shift(amax_read(r), f16);
  expo = int(r[kRecExp]);
}


// ---------------------------------------------------------------------------------
// big x small stream: the small operand S (one copy shared by every row and slice) sits in
// LDS; every thread contracts one m of the big operand X at a time (grid-stride within
// one slice; grid y/z = slices).  With scale records, X and S are multiplied by their
// power-of-two scales while loaded and the output's largest component is recorded.
template <int NK, int NN>
__global__ __launch_bounds__(kThreads) void k_stream(StreamArgs a) {
  constexpr int KS = 1 << NK, NS = 1 << NN;
  __shared__ float2 s_lds[KS * NS];
  __shared__ int64_t koff[KS];
  const int64_t sl = int64_t(blockIdx.y) + int64_t(blockIdx.z) * gridDim.y;
  if (sl >= a.nb) return;
  float sx = 1.f, ss = 1.f;
  if (a.rec_c) {
    int shx, shs, ex, es;
    rec_load(a.rec_x, a.rec_x_step, sl, false, shx, ex);
    rec_load(a.rec_s, a.rec_s_step, sl, false, shs, es);
    sx = pow2f(shx);
    ss = pow2f(shs);
    if (blockIdx.x == 0 && threadIdx.x == 0) a.rec_c[sl * a.rec_c_step + kRecExp] = uint32_t(ex + es - shx - shs);
  }
  for (int k = threadIdx.x; k < KS; k += kThreads) {
    int64_t ko = 0;
    for (int j = 0; j < NK; ++j)
      if ((k >> j) & 1) ko += int64_t(1) << a.x_kpos[j];
    koff[k] = ko;
  }
  for (int q = threadIdx.x; q < KS * NS; q += kThreads) {
    const int k = q / NS, n = q % NS;
    int so = 0;
    for (int j = 0; j < NK; ++j)
      if ((k >> j) & 1) so += 1 << a.s_kpos[j];
    for (int j = 0; j < NN; ++j)
      if ((n >> j) & 1) so += 1 << a.s_npos[j];
    const float2 v = a.S[so];
    s_lds[q] = make_float2(v.x * ss, v.y * ss);
  }
  __syncthreads();
  const int64_t per_slice = a.rows << a.n_m;
  const int64_t mmask = (int64_t(1) << a.n_m) - 1;
  float mx = 0.f;
  for (int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x; g < per_slice;
       g += int64_t(gridDim.x) * kThreads) {
    const int64_t r = g >> a.n_m, m = g & mmask;
    const int64_t xr = a.gx ? a.gx[r] : (a.x_rows == 1 ? 0 : r);
    const float2* X = a.X + sl * a.x_slice_stride + xr * a.x_row_stride;
    int64_t xo = m;
#pragma unroll
    for (int j = 0; j < NK; ++j) {
      const int p = a.x_kins[j];
      xo = ((xo >> p) << (p + 1)) | (xo & ((int64_t(1) << p) - 1));
    }
    float2 xv[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const float2 v = X[xo + koff[k]];
      xv[k] = make_float2(v.x * sx, v.y * sx);
    }
    float2 acc[NS];
#pragma unroll
    for (int n = 0; n < NS; ++n) acc[n] = make_float2(0.f, 0.f);
#pragma unroll
    for (int k = 0; k < KS; ++k) {
#pragma unroll
      for (int n = 0; n < NS; ++n) {
        const float2 sv = s_lds[k * NS + n];
        acc[n].x += xv[k].x * sv.x - xv[k].y * sv.y;
        acc[n].y += xv[k].x * sv.y + xv[k].y * sv.x;
      }
    }
    float2* C = a.C + sl * a.c_slice_stride + r * a.c_row_stride + (m << NN);
#pragma unroll
    for (int n = 0; n < NS; ++n) {
      C[n] = acc[n];
      mx = fmaxf(mx, fmaxf(fabsf(acc[n].x), fabsf(acc[n].y)));
    }
  }
  if (a.rec_c) amax_commit_wg(mx, sl, a.rec_c, a.rec_c_step);
}

// ---------------------------------------------------------------------------------
// big x small stream where the small operand differs per row (sparse-state rows) or per
// slice: each workgroup stages the small operands of its rows in LDS once (coalesced along
// each row), then every thread contracts one (row, m) item, or a 1/nsplit share of its N
// outputs, reading the small operand from LDS.  Grid: x = row chunks (or 256-item
// segments of one row when M >= 256), y/z = slices.
constexpr int kStageElems = 4096;   // complex entries of staged small operands per workgroup

template <int NK, int NN>
__global__ __launch_bounds__(kThreads) void k_stream_rows(StreamArgs a, int rw, int nsplit) {
  constexpr int KS = 1 << NK, NS = 1 << NN, E = KS * NS;
  __shared__ float2 s_lds[kStageElems];
  __shared__ int64_t koff[KS];
  __shared__ int32_t soff[E];
  const int64_t sl = int64_t(blockIdx.y) + int64_t(blockIdx.z) * gridDim.y;
  if (sl >= a.nb) return;
  float sx = 1.f, ss = 1.f;
  if (a.rec_c) {
    int shx, shs, ex, es;
    rec_load(a.rec_x, a.rec_x_step, sl, false, shx, ex);
    rec_load(a.rec_s, a.rec_s_step, sl, false, shs, es);
    sx = pow2f(shx);
    ss = pow2f(shs);
    if (blockIdx.x == 0 && threadIdx.x == 0) a.rec_c[sl * a.rec_c_step + kRecExp] = uint32_t(ex + es - shx - shs);
  }
  for (int k = threadIdx.x; k < KS; k += kThreads) {
    int64_t ko = 0;
    for (int j = 0; j < NK; ++j)
      if ((k >> j) & 1) ko += int64_t(1) << a.x_kpos[j];
    koff[k] = ko;
  }
  for (int q = threadIdx.x; q < E; q += kThreads) {
    const int k = q / NS, n = q % NS;
    int so = 0;
    for (int j = 0; j < NK; ++j)
      if ((k >> j) & 1) so += 1 << a.s_kpos[j];
    for (int j = 0; j < NN; ++j)
      if ((n >> j) & 1) so += 1 << a.s_npos[j];
    soff[q] = so;
  }
  __syncthreads();
  const int64_t M = int64_t(1) << a.n_m;
  int64_t r0, m_base, nrows;
  if (M >= kThreads) {
    const int64_t per_row = M / kThreads;
    r0 = int64_t(blockIdx.x) / per_row;
    m_base = (int64_t(blockIdx.x) % per_row) * kThreads;
    nrows = 1;
  } else {
    r0 = int64_t(blockIdx.x) * rw;
    m_base = 0;
    nrows = (a.rows - r0 < rw) ? a.rows - r0 : rw;
  }
  for (int64_t e = threadIdx.x; e < nrows * E; e += kThreads) {
    const int64_t rr = e / E, r = r0 + rr;
    const int q = int(e % E);
    const int64_t sr = a.gs ? a.gs[r] : (a.s_rows == 1 ? 0 : r);
    const float2 v = a.S[sl * a.s_slice_stride + sr * a.s_row_stride + soff[q]];
    s_lds[e] = make_float2(v.x * ss, v.y * ss);
  }
  __syncthreads();
  const int item = threadIdx.x / nsplit, part = threadIdx.x % nsplit;
  const int64_t items = (M >= kThreads) ? kThreads : nrows * M;
  float mx = 0.f;
  if (item < items) {
    int64_t rr, m;
    if (M >= kThreads) {
      rr = 0;
      m = m_base + item;
    } else {
      rr = item >> a.n_m;
      m = item & (M - 1);
    }
    const int64_t r = r0 + rr;
    const int64_t xr = a.gx ? a.gx[r] : (a.x_rows == 1 ? 0 : r);
    const float2* X = a.X + sl * a.x_slice_stride + xr * a.x_row_stride;
    int64_t xo = m;
#pragma unroll
    for (int j = 0; j < NK; ++j) {
      const int p = a.x_kins[j];
      xo = ((xo >> p) << (p + 1)) | (xo & ((int64_t(1) << p) - 1));
    }
    float2 xv[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const float2 v = X[xo + koff[k]];
      xv[k] = make_float2(v.x * sx, v.y * sx);
    }
    const float2* srow = s_lds + rr * E;
    float2* C = a.C + sl * a.c_slice_stride + r * a.c_row_stride + (m << NN);
    const int nper = NS / nsplit;
    for (int n = part * nper; n < (part + 1) * nper; ++n) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const float2 sv = srow[k * NS + n];
        acc.x += xv[k].x * sv.x - xv[k].y * sv.y;
        acc.y += xv[k].x * sv.y + xv[k].y * sv.x;
      }
      C[n] = acc;
      mx = fmaxf(mx, fmaxf(fabsf(acc.x), fabsf(acc.y)));
    }
  }
  if (a.rec_c) amax_commit_wg(mx, sl, a.rec_c, a.rec_c_step);
}

// ---------------------------------------------------------------------------------
// complex64 GEMM on v_mfma_f32_32x32x2f32
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nb) {
  // Workgroups are dealt to the 8 XCDs round-robin; renumber them so that each XCD
  // receives a contiguous range of tiles (neighbouring tiles share operand panels,
  // which then stay in that XCD's L2).
  const int64_t q = nb / 8, rem = nb % 8, x = bid % 8;
  return x * q + (x < rem ? x : rem) + bid / 8;
}

// Scatter the low `nbits` bits of x to the bit positions pos[0..nbits) (a software pdep).
// Unrolled to MAXB >= nbits iterations so that pos[] is read at constant offsets (scalar
// loads from the kernel arguments) instead of through a dynamically indexed array.
template <int MAXB>
__device__ __forceinline__ int64_t scatter_u(int64_t x, const int8_t* pos, int nbits) {
  int64_t o = 0;
#pragma unroll
  for (int j = 0; j < MAXB; ++j)
    if (j < nbits) o += ((x >> j) & 1) << pos[j];
  return o;
}

__device__ __forceinline__ float2 keep_if(float2 v, uint32_t mask) {
  uint2 u = __builtin_bit_cast(uint2, v);
  u.x &= mask;
  u.y &= mask;
  return __builtin_bit_cast(float2, u);
}

// Tile bookkeeping shared by the GEMM kernels: which output tile, slice, row and K range
// this workgroup owns, the operand bases of the tile corner, and for every load slot of
// this thread its scattered element offset inside the tile.  Tile sizes divide a label
// group whenever the group is larger than the tile, so the corner bits and the in-tile
// bits never overlap.
//
// The scattered offset of a K tile is a sum over 6-bit digits of the tile index (at most
// kKLevels digits: K <= 2^(4 + 6 kKLevels), checked when the plan is compiled); entry d of
// the level-l table holds the offset of digit value d at level l.  The tables sit either
// in LDS (LDS_TAB) or one entry per lane in registers, read with readlane.  Offsets within
// one operand row fit in 31 bits (also checked when the plan is compiled).
constexpr int kKLevels = 4;

// Operand scales of a GEMM for slice copy sl from the records of A and B; the workgroup
// that owns the slice's first tile (`writer`) records C's exponent.
__device__ __forceinline__ void rec_scales(const GemmArgs& a, int64_t sl, bool f16, bool writer,
                                           float& sa, float& sb) {
  int sha, shb, ea, eb;
  rec_load(a.rec_a, a.rec_a_step, sl, f16, sha, ea);
  rec_load(a.rec_b, a.rec_b_step, sl, f16, shb, eb);
  sa = pow2f(sha);
  sb = pow2f(shb);
  if (writer && threadIdx.x == 0) a.rec_c[sl * a.rec_c_step + kRecExp] = uint32_t(ea + eb - sha - shb);
}

template <int BM, int BN, int BK, bool A_MFAST, bool B_NFAST, bool LDS_TAB, int NT = kThreads>
struct GemmTile {
  static constexpr int LBM = (BM == 256) ? 8 : (BM == 128) ? 7 : (BM == 64 ? 6 : 5);
  static constexpr int LBN = (BN == 128) ? 7 : (BN == 64 ? 6 : (BN == 32 ? 5 : (BN == 16 ? 4 : 3)));
  static constexpr int LBK = (BK == 16) ? 4 : (BK == 32 ? 5 : 3);
  static constexpr int A_LD = BM * BK / NT;
  static constexpr int B_LD = (BK * BN + NT - 1) / NT;
  static constexpr int kLev = kKLevels;
  static constexpr int kTab = 2 * kLev * 64;   // LDS table entries (A levels, then B levels)

  const float2* A;
  const float2* B;
  int64_t M, N, m0, n0, k_begin, k_end, zr, sl, r;
  int64_t stk_start, stk_count;   // stacked rows of this tile's 128-row block
  int ks, nlev;
  int32_t ka_t[LDS_TAB ? 1 : kLev], kb_t[LDS_TAB ? 1 : kLev];
  const int32_t* tab;
  int32_t a_off[A_LD], b_off[B_LD];
  uint32_t in_bits;   // bit i: A slot i in range; bit A_LD + i: B slot i in range
  uint32_t full_bits; // in_bits of an interior tile (every existing slot in range)

  // (row, col) of A slot i and (k, n) of B slot i inside the tile.  Consecutive lanes take
  // consecutive addresses of the operand's fastest index (coalesced loads); when that index
  // is m (n), a thread's slots are consecutive k of one row (column).
  __device__ __forceinline__ static int a_row(int i) {
    const int q = threadIdx.x + i * NT;
    return A_MFAST ? int(threadIdx.x) % BM : q / BK;
  }
  __device__ __forceinline__ static int a_col(int i) {
    const int q = threadIdx.x + i * NT;
    return A_MFAST ? (int(threadIdx.x) / BM) * A_LD + i : q % BK;
  }
  __device__ __forceinline__ static int b_kr(int i) {
    const int q = threadIdx.x + i * NT;
    return B_NFAST ? (BK * BN >= NT ? (int(threadIdx.x) / BN) * B_LD + i : q / BN) : q % BK;
  }
  __device__ __forceinline__ static int b_n(int i) {
    const int q = threadIdx.x + i * NT;
    return B_NFAST ? (BK * BN >= NT ? int(threadIdx.x) % BN : q % BN) : q / BK;
  }
  __device__ __forceinline__ static bool b_slot(int i) {
    return BK * BN % NT == 0 || threadIdx.x + i * NT < BK * BN;
  }

  __device__ __forceinline__ bool init(const GemmArgs& a, int32_t* lds_tab = nullptr) {
    M = a.M;
    N = a.N;
    const int64_t tiles_m = (M + BM - 1) / BM;
    const int64_t tiles_n = (N + BN - 1) / BN;
    const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
    if (tile >= tiles_m * tiles_n) return false;
    // grouped numbering: consecutive tiles (one XCD's range after the remap) cover a block
    // of group_m tile rows by several tile columns, so they share A and B panels in L2
    int64_t tm, tn;
    if (a.group_m > 1) {
      const int64_t gm = a.group_m;
      const int64_t per_group = gm * tiles_n, g = tile / per_group, first = g * gm;
      const int64_t gsize = (tiles_m - first < gm) ? tiles_m - first : gm;
      tm = first + (tile % per_group) % gsize;
      tn = (tile % per_group) / gsize;
    } else {
      tm = tile % tiles_m;
      tn = tile / tiles_m;
    }
    const int64_t z = int64_t(blockIdx.y) + int64_t(blockIdx.z) * gridDim.y;
    zr = z / a.k_splits;      // slice * rows + row
    ks = int(z % a.k_splits);
    if (zr >= a.rows * a.nb) return false;
    sl = zr / a.rows;
    r = zr - sl * a.rows;
    m0 = tm * BM;
    n0 = tn * BN;
    const int64_t mloc_mask = (int64_t(1) << a.nm) - 1;
    if (a.stk) {
      const int32_t* e = a.stk + 3 * (m0 >> 7);
      stk_start = e[0];
      stk_count = e[1];
      A = a.A + sl * a.a_slice_stride;
      B = a.B + sl * a.b_slice_stride + int64_t(e[2]) * a.b_row_stride +
          scatter_u<kMaxRank>(n0, a.b_npos, a.nn);
    } else {
      const int64_t ar = a.ga ? a.ga[r] : (a.a_rows == 1 ? 0 : r);
      const int64_t br = a.gb ? a.gb[r] : (a.b_rows == 1 ? 0 : r);
      A = a.A + sl * a.a_slice_stride + ar * a.a_row_stride +
          (a.fold ? (m0 >> a.nm) * a.fold_stride : 0) +
          scatter_u<kMaxRank>(m0 & mloc_mask, a.a_mpos, a.nm);
      B = a.B + sl * a.b_slice_stride + br * a.b_row_stride + scatter_u<kMaxRank>(n0, a.b_npos, a.nn);
    }
    k_begin = int64_t(ks) * a.k_chunk;
    k_end = (k_begin + a.k_chunk < a.K) ? k_begin + a.k_chunk : a.K;
    nlev = a.nk > LBK ? (a.nk - LBK + 5) / 6 : 0;
    if (LDS_TAB && nlev > 0) {
      for (int e = threadIdx.x; e < kTab; e += NT) {
        const int op = e / (kLev * 64), l = (e / 64) % kLev, d = e % 64;
        const int lo = LBK + 6 * l;
        const int nb = a.nk - lo < 0 ? 0 : (a.nk - lo > 6 ? 6 : a.nk - lo);
        lds_tab[e] = int32_t(scatter_u<6>(d, (op ? a.b_kpos : a.a_kpos) + lo, nb));
      }
      tab = lds_tab;
    } else {
      const int lane = threadIdx.x & 63;
#pragma unroll
      for (int l = 0; l < kLev; ++l) {
        const int lo = LBK + 6 * l;
        const int nb = a.nk - lo < 0 ? 0 : (a.nk - lo > 6 ? 6 : a.nk - lo);
        ka_t[l] = int32_t(scatter_u<6>(lane, a.a_kpos + lo, nb));
        kb_t[l] = int32_t(scatter_u<6>(lane, a.b_kpos + lo, nb));
      }
    }
    const int nbm = a.nm < LBM ? a.nm : LBM, nbk = a.nk < LBK ? a.nk : LBK;
    const int nbn = a.nn < LBN ? a.nn : LBN;
    in_bits = 0;
    full_bits = (1u << A_LD) - 1;
#pragma unroll
    for (int i = 0; i < B_LD; ++i) full_bits |= uint32_t(b_slot(i)) << (A_LD + i);
#pragma unroll
    for (int i = 0; i < A_LD; ++i) {
      const int row = a_row(i), col = a_col(i);
      if (a.stk) {
        // stacked: slot row -> (output row, m inside it); offsets from the slice base
        const int64_t w = (m0 & 127) + row, rr = w >> a.nm, mm = w & mloc_mask;
        const bool in = rr < stk_count;
        const int64_t cr = in ? a.perm[stk_start + rr] : 0;
        const int64_t ar = a.ga ? a.ga[cr] : (a.a_rows == 1 ? 0 : cr);
        a_off[i] = in ? int32_t(ar * a.a_row_stride + scatter_u<7>(mm, a.a_mpos, a.nm) +
                                scatter_u<LBK>(col, a.a_kpos, nbk))
                      : 0;
        in_bits |= uint32_t(in) << i;
      } else {
        const bool in = (m0 + row < M);
        // out-of-range slots read the tile corner (always valid) and are masked to zero
        a_off[i] = in ? int32_t(scatter_u<LBM>(row, a.a_mpos, nbm) + scatter_u<LBK>(col, a.a_kpos, nbk)) : 0;
        in_bits |= uint32_t(in) << i;
      }
    }
#pragma unroll
    for (int i = 0; i < B_LD; ++i) {
      const int kr = b_kr(i), n = b_n(i);
      const bool in = b_slot(i) && (n0 + n < N);
      b_off[i] = in ? int32_t(scatter_u<LBK>(kr, a.b_kpos, nbk) + scatter_u<LBN>(n, a.b_npos, nbn)) : 0;
      in_bits |= uint32_t(in) << (A_LD + i);
    }
    if (LDS_TAB && nlev > 0) __syncthreads();
    return true;
  }

  // global -> registers.  `valid` receives the in-range bits of the slots; they are applied
  // (masked to zero) when the registers are written to LDS, so no wait is forced here.
  __device__ __forceinline__ void load(const GemmArgs& a, int64_t k0, float2* ra, float2* rb,
                                       uint32_t& valid) const {
    const int64_t kt = k0 >> LBK;
    int32_t oa = 0, ob = 0;
#pragma unroll
    for (int l = 0; l < kLev; ++l)
      if (l < nlev) {
        const int d = int((kt >> (6 * l)) & 63);
        if (LDS_TAB) {
          oa += tab[l * 64 + d];
          ob += tab[(kLev + l) * 64 + d];
        } else {
          oa += __builtin_amdgcn_readlane(ka_t[LDS_TAB ? 0 : l], d);
          ob += __builtin_amdgcn_readlane(kb_t[LDS_TAB ? 0 : l], d);
        }
      }
    const float2* __restrict__ Ak = A + oa;
    const float2* __restrict__ Bk = B + ob;
    const int64_t kl = k_end - k0;
    if (kl >= BK) {
#pragma unroll
      for (int i = 0; i < A_LD; ++i) ra[i] = Ak[a_off[i]];
#pragma unroll
      for (int i = 0; i < B_LD; ++i) rb[i] = Bk[b_off[i]];
      valid = in_bits;
    } else {
      uint32_t v = in_bits;
#pragma unroll
      for (int i = 0; i < A_LD; ++i) {
        const bool ok = a_col(i) < kl;
        ra[i] = Ak[ok ? a_off[i] : 0];
        if (!ok) v &= ~(1u << i);
      }
#pragma unroll
      for (int i = 0; i < B_LD; ++i) {
        const bool ok = b_kr(i) < kl;
        rb[i] = Bk[ok ? b_off[i] : 0];
        if (!ok) v &= ~(1u << (A_LD + i));
      }
      valid = v;
    }
  }

  // the workgroup of the slice's first tile, row and split (records C's exponent)
  __device__ __forceinline__ bool first_of_slice() const {
    return m0 == 0 && n0 == 0 && r == 0 && ks == 0;
  }

  // zero the slots that are out of range
  __device__ __forceinline__ static void apply(uint32_t valid, float2* ra, float2* rb) {
#pragma unroll
    for (int i = 0; i < A_LD; ++i) ra[i] = keep_if(ra[i], ((valid >> i) & 1) ? ~0u : 0u);
#pragma unroll
    for (int i = 0; i < B_LD; ++i) rb[i] = keep_if(rb[i], ((valid >> (A_LD + i)) & 1) ? ~0u : 0u);
  }

  // multiply the staged values by the operands' power-of-two scales (exact)
  __device__ __forceinline__ static void scale(float sa, float sb, float2* ra, float2* rb) {
#pragma unroll
    for (int i = 0; i < A_LD; ++i) ra[i] = make_float2(ra[i].x * sa, ra[i].y * sa);
#pragma unroll
    for (int i = 0; i < B_LD; ++i) rb[i] = make_float2(rb[i].x * sb, rb[i].y * sb);
  }

  __device__ __forceinline__ float* out(const GemmArgs& a) const {
    return (a.k_splits > 1)
               ? reinterpret_cast<float*>(a.partial + (int64_t(ks) * a.rows * a.nb + zr) * M * N)
               : reinterpret_cast<float*>(a.C + sl * a.c_slice_stride + r * a.c_row_stride);
  }

  // first float of output row `row` of this tile (plain, split-K partial or stacked), or
  // nullptr when that row lies outside the output
  __device__ __forceinline__ float* row_ptr(const GemmArgs& a, int row) const {
    if (a.stk) {
      const int64_t w = (m0 & 127) + row, rr = w >> a.nm;
      if (rr >= stk_count) return nullptr;
      const int64_t cr = a.perm[stk_start + rr];
      return reinterpret_cast<float*>(a.C + sl * a.c_slice_stride) +
             (cr * a.c_row_stride + (w & ((int64_t(1) << a.nm) - 1)) * N) * 2;
    }
    if (m0 + row >= M) return nullptr;
    return out(a) + (m0 + row) * N * 2;
  }

  // largest |value| among this lane's accumulators: entries outside the output hold exact
  // zeros (their operand slots were zeroed when staged), so no bounds are needed
  template <int UM, int UN>
  __device__ __forceinline__ static float acc_absmax(const f32x16 (&acc)[UM][UN]) {
    float m = 0.f;
#pragma unroll
    for (int i = 0; i < UM; ++i)
#pragma unroll
      for (int j = 0; j < UN; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) m = fmaxf(m, fabsf(acc[i][j][v]));
    return m;
  }

  // 32x32 accumulator layout: column = lane % 32, row = 8 (v/4) + 4 (lane/32) + v%4; the
  // real column j is complex column j/2, real part for even j
  template <int UM, int UN>
  __device__ __forceinline__ void store_acc(const GemmArgs& a, const f32x16 (&acc)[UM][UN],
                                            int wm_base, int wn_base) const {
    const int lane = threadIdx.x & 63, half = lane >> 5, j32 = lane & 31;
    if (a.stk) {
      // stacked rows: each output row of the tile maps to (row of C, m inside it)
      float* cb = reinterpret_cast<float*>(a.C + sl * a.c_slice_stride);
      const int64_t mmask = (int64_t(1) << a.nm) - 1;
#pragma unroll
      for (int i = 0; i < UM; ++i)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = wm_base + i * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
          const int64_t w = (m0 & 127) + row, rr = w >> a.nm;
          if (rr >= stk_count) continue;
          const int64_t cr = a.perm[stk_start + rr];
          float* orow = cb + (cr * a.c_row_stride + (w & mmask) * N) * 2;
#pragma unroll
          for (int j = 0; j < UN; ++j) {
            const int64_t np = n0 + wn_base + j * 16 + (j32 >> 1);
            if (np < N) orow[np * 2 + (j32 & 1)] = acc[i][j][v];
          }
        }
      return;
    }
    float* o = out(a);
#pragma unroll
    for (int i = 0; i < UM; ++i)
#pragma unroll
      for (int j = 0; j < UN; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = wm_base + i * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
          const int64_t m = m0 + row;
          const int64_t np = n0 + wn_base + j * 16 + (j32 >> 1);
          if (m < M && np < N) o[(m * N + np) * 2 + (j32 & 1)] = acc[i][j][v];
        }
  }
};

template <int WAVES_M, int WAVES_N, int UM, int UN, int BK, bool A_MFAST, bool B_NFAST>
__global__ __launch_bounds__(WAVES_M * WAVES_N * 64) __attribute__((amdgpu_waves_per_eu(WAVES_M * WAVES_N == 4 ? 3 : 2))) void k_gemm(GemmArgs a) {
  constexpr int NT = WAVES_M * WAVES_N * 64;   // four or eight waves
  static_assert(NT == 256 || NT == 512, "four or eight waves per workgroup");
  constexpr int BM = WAVES_M * UM * 32;
  constexpr int BN = WAVES_N * UN * 16;
  using Tile = GemmTile<BM, BN, BK, A_MFAST, B_NFAST, true, NT>;
  constexpr int A_LD = Tile::A_LD, B_LD = Tile::B_LD;
  constexpr int AS = 2 * BK + 2;       // floats per LDS row of A (m-major)
  constexpr int BS = 2 * BN;           // floats per LDS row of B (k-major; reads are broadcasts)
  constexpr int A_STAGE = BM * AS, B_STAGE = BK * BS;
  // two LDS stages: stage t is read while the tile of stage t+1 is written
  __shared__ float As[2 * A_STAGE];
  __shared__ float Bs[2 * B_STAGE];
  __shared__ int32_t ktab[Tile::kTab];

  Tile t;
  if (!t.init(a, ktab)) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave % WAVES_M, wn = wave / WAVES_M;
  float sa = 1.f, sb = 1.f;
  bool scaled = false;

  f32x16 acc[UM][UN];
#pragma unroll
  for (int i = 0; i < UM; ++i)
#pragma unroll
    for (int j = 0; j < UN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  float2 ra[A_LD], rb[B_LD];
  uint32_t valid = 0;
  auto store = [&](int stage) {
    if (valid != t.full_bits) Tile::apply(valid, ra, rb);
    if (scaled) Tile::scale(sa, sb, ra, rb);
    float* as = As + stage * A_STAGE;
    float* bs = Bs + stage * B_STAGE;
#pragma unroll
    for (int i = 0; i < A_LD; ++i)
      *reinterpret_cast<float2*>(&as[Tile::a_row(i) * AS + 2 * Tile::a_col(i)]) = ra[i];
#pragma unroll
    for (int i = 0; i < B_LD; ++i)
      if (BK * BN % NT == 0 || threadIdx.x + i * NT < BK * BN)
        *reinterpret_cast<float2*>(&bs[Tile::b_kr(i) * BS + 2 * Tile::b_n(i)]) = rb[i];
  };

  const int half = lane >> 5;          // 0: lanes carry Re(A); 1: lanes carry Im(A)
  const int j32 = lane & 31;
  const int bc = j32 & 1;              // output column parity: 0 = real part, 1 = imaginary
  // real embedding of B: rows (Re k, Im k) x columns (Re n, Im n) -> this lane takes the
  // imaginary part when its (row, column) parities differ, negated for (Im k, Re n)
  const bool b_take_im = (half != bc);
  const float b_sign = (half == 1 && bc == 0) ? -1.f : 1.f;
  int a_rd[UM], b_rd[UN];
#pragma unroll
  for (int i = 0; i < UM; ++i) a_rd[i] = (wm * UM * 32 + i * 32 + j32) * AS + half;
#pragma unroll
  for (int j = 0; j < UN; ++j) b_rd[j] = 2 * (wn * UN * 16 + j * 16 + (j32 >> 1));

  int stage = 0;
  if (t.k_begin < t.k_end) t.load(a, t.k_begin, ra, rb, valid);
  if (a.rec_c) {   // the records are read while the first tile's loads are in flight
    rec_scales(a, t.sl, false, t.first_of_slice(), sa, sb);
    scaled = (sa != 1.f) || (sb != 1.f);
  }
  if (t.k_begin < t.k_end) store(0);
  __syncthreads();
  for (int64_t k0 = t.k_begin; k0 < t.k_end; k0 += BK) {
    const bool more = k0 + BK < t.k_end;
    if (more) t.load(a, k0 + BK, ra, rb, valid);
    const float* as = As + stage * A_STAGE;
    const float* bs = Bs + stage * B_STAGE;
    // fragments double-buffered in registers: step kk+1 is read from LDS before the
    // matrix-core instructions of step kk are issued
    float af[2][UM];
    float2 bv[2][UN];
#pragma unroll
    for (int i = 0; i < UM; ++i) af[0][i] = as[a_rd[i]];
#pragma unroll
    for (int j = 0; j < UN; ++j) bv[0][j] = *reinterpret_cast<const float2*>(&bs[b_rd[j]]);
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      const int cur = kk & 1, nxt = cur ^ 1;
      if (kk + 1 < BK) {
#pragma unroll
        for (int i = 0; i < UM; ++i) af[nxt][i] = as[a_rd[i] + 2 * (kk + 1)];
#pragma unroll
        for (int j = 0; j < UN; ++j)
          bv[nxt][j] = *reinterpret_cast<const float2*>(&bs[(kk + 1) * BS + b_rd[j]]);
      }
      float bf[UN];
#pragma unroll
      for (int j = 0; j < UN; ++j) bf[j] = (b_take_im ? bv[cur][j].y : bv[cur][j].x) * b_sign;
      // keep the reads of step kk+1 ahead of this step's matrix instructions
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < UM; ++i)
#pragma unroll
        for (int j = 0; j < UN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[cur][i], bf[j], acc[i][j], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
      // the next K tile goes to the other LDS stage halfway through this one, so that
      // the writes overlap the matrix instructions instead of preceding the barrier
      if (kk == BK / 2 && more) store(stage ^ 1);
    }
    __syncthreads();
    stage ^= 1;
  }
  if (a.rec_c && a.k_splits == 1)
    amax_commit_wg(Tile::template acc_absmax<UM, UN>(acc), t.sl, a.rec_c, a.rec_c_step);
  t.template store_acc<UM, UN>(a, acc, wm * UM * 32, wn * UN * 16);
}

// ---------------------------------------------------------------------------------
// complex64 GEMM for N <= 8 on v_mfma_f32_16x16x4f32: the same real embedding with 16 real
// output columns (8 complex), each instruction consuming two complex k, so narrow steps do
// not pay for a 32-column MFMA tile.  Tile 128 x 8 complex: four waves of 32 rows, two
// 16-row MFMA tiles each.  Lane layout of the 16x16x4 operands: A row = lane % 16, real k =
// lane / 16; B real k = lane / 16, column = lane % 16; D rows 4 (lane / 16) + v, column
// lane % 16 (real column j is complex column j / 2, real part for even j).
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <bool A_MFAST, bool B_NFAST>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_gemm_n8(GemmArgs a) {
  constexpr int BM = 128, BN = 8, BK = 16, UM = 2;
  using Tile = GemmTile<BM, BN, BK, A_MFAST, B_NFAST, true>;
  constexpr int A_LD = Tile::A_LD, B_LD = Tile::B_LD;
  constexpr int AS = 2 * BK + 2, BS = 2 * BN;
  constexpr int A_STAGE = BM * AS, B_STAGE = BK * BS;
  __shared__ float As[2 * A_STAGE];
  __shared__ float Bs[2 * B_STAGE];
  __shared__ int32_t ktab[Tile::kTab];

  Tile t;
  if (!t.init(a, ktab)) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float sa = 1.f, sb = 1.f;
  bool scaled = false;
  f32x4 acc[UM];
#pragma unroll
  for (int i = 0; i < UM; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[i][v] = 0.f;

  float2 ra[A_LD], rb[B_LD];
  uint32_t valid = 0;
  auto store = [&](int stage) {
    if (valid != t.full_bits) Tile::apply(valid, ra, rb);
    if (scaled) Tile::scale(sa, sb, ra, rb);
    float* as = As + stage * A_STAGE;
    float* bs = Bs + stage * B_STAGE;
#pragma unroll
    for (int i = 0; i < A_LD; ++i)
      *reinterpret_cast<float2*>(&as[Tile::a_row(i) * AS + 2 * Tile::a_col(i)]) = ra[i];
#pragma unroll
    for (int i = 0; i < B_LD; ++i)
      if (Tile::b_slot(i))
        *reinterpret_cast<float2*>(&bs[Tile::b_kr(i) * BS + 2 * Tile::b_n(i)]) = rb[i];
  };

  const int r16 = lane & 15, q = lane >> 4;     // q: real k within the instruction
  const int part = q & 1, col = r16, bc = col & 1;
  const bool b_take_im = (part != bc);
  const float b_sign = (part == 1 && bc == 0) ? -1.f : 1.f;
  int a_rd[UM];
#pragma unroll
  for (int i = 0; i < UM; ++i) a_rd[i] = (wave * 32 + i * 16 + r16) * AS + q;
  const int b_rd = (q >> 1) * BS + 2 * (col >> 1);

  int stage = 0;
  if (t.k_begin < t.k_end) t.load(a, t.k_begin, ra, rb, valid);
  if (a.rec_c) {
    rec_scales(a, t.sl, false, t.first_of_slice(), sa, sb);
    scaled = (sa != 1.f) || (sb != 1.f);
  }
  if (t.k_begin < t.k_end) store(0);
  __syncthreads();
  for (int64_t k0 = t.k_begin; k0 < t.k_end; k0 += BK) {
    const bool more = k0 + BK < t.k_end;
    if (more) t.load(a, k0 + BK, ra, rb, valid);
    const float* as = As + stage * A_STAGE;
    const float* bs = Bs + stage * B_STAGE;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      float af[UM];
#pragma unroll
      for (int i = 0; i < UM; ++i) af[i] = as[a_rd[i] + 2 * kk];
      const float2 bv = *reinterpret_cast<const float2*>(&bs[kk * BS + b_rd]);
      const float bf = (b_take_im ? bv.y : bv.x) * b_sign;
#pragma unroll
      for (int i = 0; i < UM; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf, acc[i], 0, 0, 0);
    }
    if (more) store(stage ^ 1);
    __syncthreads();
    stage ^= 1;
  }
  const int64_t np = t.n0 + (col >> 1);
  float mx = 0.f;
#pragma unroll
  for (int i = 0; i < UM; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float* o = t.row_ptr(a, wave * 32 + i * 16 + 4 * q + v);
      if (o && np < t.N) {
        o[np * 2 + bc] = acc[i][v];
        mx = fmaxf(mx, fabsf(acc[i][v]));
      }
    }
  if (a.rec_c && a.k_splits == 1) amax_commit_wg(mx, t.sl, a.rec_c, a.rec_c_step);
}

// ---------------------------------------------------------------------------------
// complex64 products with a short contraction (K = 2^NK <= 16) and a wide output,
// C[r][m][n] = sum_k A[m,k] B[k,n], on the vector ALUs.  Such steps are bound by writing
// C (up to 8 GiB per slice): a workgroup owns kOuterCols columns x kOuterRows rows of one
// output row; each thread keeps the KS x 2 values of B for two consecutive columns in
// registers, the workgroup stages kOuterStage rows of A at a time in LDS (read as
// broadcasts), and every thread writes its two complex outputs of a row as one 16-byte
// store, consecutive lanes at consecutive addresses.  Operands are read in their stored
// label order (scattered offsets, as in the GEMM); rows may be folded into M (fold) but
// not stacked; no split-K.
constexpr int kOuterCols = 512, kOuterRows = 256, kOuterStage = 64;

template <int NK>
__global__ __launch_bounds__(kThreads) void k_gemm_outer(GemmArgs a) {
  constexpr int KS = 1 << NK;
  __shared__ float2 As[kOuterStage * KS];
  const int64_t M = a.M, N = a.N;
  const int cols = N < kOuterCols ? int(N) : kOuterCols;   // columns of this workgroup
  const int tpr = cols / 2;                                 // threads per output row
  const int rpp = kThreads / tpr;                           // output rows per pass
  const int64_t col_blocks = N / cols;
  const int64_t mrows = M < kOuterRows ? M : kOuterRows;
  const int64_t cb = int64_t(blockIdx.x) % col_blocks, mb = int64_t(blockIdx.x) / col_blocks;
  const int64_t n0 = cb * cols, mw0 = mb * mrows;
  const int64_t z = int64_t(blockIdx.y) + int64_t(blockIdx.z) * gridDim.y;
  if (z >= a.rows * a.nb) return;
  const int64_t sl = z / a.rows, r = z - sl * a.rows;
  const int64_t ar = a.ga ? a.ga[r] : (a.a_rows == 1 ? 0 : r);
  const int64_t br = a.gb ? a.gb[r] : (a.b_rows == 1 ? 0 : r);
  const float2* A = a.A + sl * a.a_slice_stride + ar * a.a_row_stride;
  const float2* B = a.B + sl * a.b_slice_stride + br * a.b_row_stride;
  float2* C = a.C + sl * a.c_slice_stride + r * a.c_row_stride;
  float sa = 1.f, sb = 1.f;
  if (a.rec_c) {
    int sha, shb, ea, eb;
    rec_load(a.rec_a, a.rec_a_step, sl, false, sha, ea);
    rec_load(a.rec_b, a.rec_b_step, sl, false, shb, eb);
    sa = pow2f(sha);
    sb = pow2f(shb);
    if (blockIdx.x == 0 && r == 0 && threadIdx.x == 0)
      a.rec_c[sl * a.rec_c_step + kRecExp] = uint32_t(ea + eb - sha - shb);
  }
  // B: this thread's two columns, every k
  const int tc = threadIdx.x % tpr, tr = threadIdx.x / tpr;
  const int64_t n = n0 + 2 * tc;
  float2 b0[KS], b1[KS];
  {
    const int64_t o0 = scatter_u<kMaxRank>(n, a.b_npos, a.nn), o1 = scatter_u<kMaxRank>(n + 1, a.b_npos, a.nn);
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int64_t ko = scatter_u<NK>(k, a.b_kpos, NK);
      const float2 v0 = B[o0 + ko], v1 = B[o1 + ko];
      b0[k] = make_float2(v0.x * sb, v0.y * sb);
      b1[k] = make_float2(v1.x * sb, v1.y * sb);
    }
  }
  const int64_t mloc_mask = (int64_t(1) << a.nm) - 1;
  const int64_t m_end = (mw0 + mrows < M) ? mw0 + mrows : M;
  float mx = 0.f;
  for (int64_t m0 = mw0; m0 < m_end; m0 += kOuterStage) {
    const int stage_rows = int(m_end - m0 < kOuterStage ? m_end - m0 : kOuterStage);
    __syncthreads();   // the previous stage has been read
    for (int e = threadIdx.x; e < stage_rows * KS; e += kThreads) {
      const int i = e / KS, k = e % KS;
      const int64_t m = m0 + i;
      const int64_t mo = (a.fold ? (m >> a.nm) * a.fold_stride : 0) +
                         scatter_u<kMaxRank>(m & mloc_mask, a.a_mpos, a.nm);
      const float2 v = A[mo + scatter_u<NK>(k, a.a_kpos, NK)];
      As[e] = make_float2(v.x * sa, v.y * sa);
    }
    __syncthreads();
    for (int i = tr; i < stage_rows; i += rpp) {
      float c0r = 0.f, c0i = 0.f, c1r = 0.f, c1i = 0.f;
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const float2 av = As[i * KS + k];
        c0r += av.x * b0[k].x - av.y * b0[k].y;
        c0i += av.x * b0[k].y + av.y * b0[k].x;
        c1r += av.x * b1[k].x - av.y * b1[k].y;
        c1i += av.x * b1[k].y + av.y * b1[k].x;
      }
      mx = fmaxf(mx, fmaxf(fmaxf(fabsf(c0r), fabsf(c0i)), fmaxf(fabsf(c1r), fabsf(c1i))));
      float4* dst = reinterpret_cast<float4*>(C + (m0 + i) * N + n);
      *dst = make_float4(c0r, c0i, c1r, c1i);
    }
  }
  if (a.rec_c) amax_commit_wg(mx, sl, a.rec_c, a.rec_c_step);
}

// Sparse-state steps whose rows each hold a small product (M x N <= 128, N <= 4, M >= 8)
// over a long contraction (64 <= K <= 4096), e.g. 16384 rows of 32 x 2 x 512: the tiles of
// the matrix-core kernels would be mostly empty and their loads mostly masked.  One wave
// per (slice, row): lane l takes k = 16 k_hi + l % 16 and the rows m = 4 m_hi + l / 16, so
// one load instruction reads 16 consecutive k of 4 rows of A (whole 128-byte pieces when
// A's lowest index bits are k bits); each lane accumulates its share of k for its M/4 x N
// outputs in registers, and the 16 lanes of one row group are summed with cross-lane
// shuffles.  Offsets of A's and B's k indices sit in LDS tables (dynamic shared memory,
// 8 bytes per k), those of m and n in small static ones.  Operands are rescaled by their
// records while loaded, as everywhere; the output's largest component is committed per
// wave (a workgroup's waves may belong to two slices).
template <int MH, int NN>
__global__ __launch_bounds__(kThreads) void k_gemm_rows_narrow(GemmArgs a) {
  constexpr int NS = 1 << NN, MR = 4 * MH;
  extern __shared__ int32_t ktabs[];   // [K] A offsets of k, then [K] B offsets of k
  __shared__ int32_t moff[MR], noff[NS];
  const int K = int(a.K);
  int32_t* koa = ktabs;
  int32_t* kob = ktabs + K;
  for (int k = threadIdx.x; k < K; k += kThreads) {
    koa[k] = int32_t(scatter_u<kMaxRank>(k, a.a_kpos, a.nk));
    kob[k] = int32_t(scatter_u<kMaxRank>(k, a.b_kpos, a.nk));
  }
  for (int m = threadIdx.x; m < MR; m += kThreads) moff[m] = int32_t(scatter_u<kMaxRank>(m, a.a_mpos, a.nm));
  for (int n = threadIdx.x; n < NS; n += kThreads) noff[n] = int32_t(scatter_u<kMaxRank>(n, a.b_npos, a.nn));
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kl = lane & 15, ms = lane >> 4;
  const int64_t z = (int64_t(blockIdx.x) + int64_t(blockIdx.y) * gridDim.x) * 4 + wave;
  float mx = 0.f;
  if (z < a.rows * a.nb) {
    const int64_t sl = z / a.rows, r = z - sl * a.rows;
    const int64_t ar = a.ga ? a.ga[r] : (a.a_rows == 1 ? 0 : r);
    const int64_t br = a.gb ? a.gb[r] : (a.b_rows == 1 ? 0 : r);
    const float2* A = a.A + sl * a.a_slice_stride + ar * a.a_row_stride;
    const float2* B = a.B + sl * a.b_slice_stride + br * a.b_row_stride;
    float sa = 1.f, sb = 1.f;
    if (a.rec_c) {
      int sha, shb, ea, eb;
      rec_load(a.rec_a, a.rec_a_step, sl, false, sha, ea);
      rec_load(a.rec_b, a.rec_b_step, sl, false, shb, eb);
      sa = pow2f(sha);
      sb = pow2f(shb);
      if (r == 0 && lane == 0) a.rec_c[sl * a.rec_c_step + kRecExp] = uint32_t(ea + eb - sha - shb);
    }
    int32_t mo[MH];
#pragma unroll
    for (int mh = 0; mh < MH; ++mh) mo[mh] = moff[4 * mh + ms];
    float2 acc[MH][NS];
#pragma unroll
    for (int mh = 0; mh < MH; ++mh)
#pragma unroll
      for (int n = 0; n < NS; ++n) acc[mh][n] = make_float2(0.f, 0.f);
#pragma unroll 2
    for (int k = kl; k < K; k += 16) {
      const int32_t ka = koa[k], kb = kob[k];
      float2 bv[NS];
#pragma unroll
      for (int n = 0; n < NS; ++n) {
        const float2 v = B[kb + noff[n]];
        bv[n] = make_float2(v.x * sb, v.y * sb);
      }
#pragma unroll
      for (int mh = 0; mh < MH; ++mh) {
        const float2 v = A[mo[mh] + ka];
        const float2 av = make_float2(v.x * sa, v.y * sa);
#pragma unroll
        for (int n = 0; n < NS; ++n) {
          acc[mh][n].x += av.x * bv[n].x - av.y * bv[n].y;
          acc[mh][n].y += av.x * bv[n].y + av.y * bv[n].x;
        }
      }
    }
    float2* C = a.C + sl * a.c_slice_stride + r * a.c_row_stride;
#pragma unroll
    for (int mh = 0; mh < MH; ++mh)
#pragma unroll
      for (int n = 0; n < NS; ++n) {
        float re = acc[mh][n].x, im = acc[mh][n].y;
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
          re += __shfl_xor(re, off);
          im += __shfl_xor(im, off);
        }
        if (kl == 0) {
          C[(4 * mh + ms) * NS + n] = make_float2(re, im);
          mx = fmaxf(mx, fmaxf(fabsf(re), fabsf(im)));
        }
      }
  }
  // the four waves of a workgroup may hold rows of two slices: one commit per wave
  if (a.rec_c && z < a.rows * a.nb) amax_commit(mx, z / a.rows, a.rec_c, a.rec_c_step);
}

// The same short-K product on the FP32 matrix cores, for K = 2^NK = 16 and N >= 64 JB,
// where the vector form above is bound by its 4 K FMAs per complex output (64 at K = 16, at
// half the FP32 rate without packed instructions) rather than by writing C.  A workgroup
// owns 64 JB columns x a range of rows set by the launch (the grid's row blocks split M);
// wave w takes 16 JB complex columns as JB 32 x 32 real blocks of v_mfma_f32_32x32x2f32
// (JB = 4: 2 waves per SIMD), each instruction consuming one complex k through
// the real embedding of B ([[Re, Im], [-Im, Re]], as in k_gemm).  The B fragments of every
// k stay in registers; 32 rows of A at a time are staged in LDS (two buffers, so the next
// rows are loaded while the current ones feed the matrix cores).  Each wave passes its
// 32 x 128 real results through its own LDS patch (row stride 136 floats: the accumulator
// writes, rows r and r + 4 per instruction, and the 16-byte reads, 64 consecutive floats
// per 16 lanes, are free of bank conflicts on a 64-bank LDS) and writes every row's 512
// contiguous bytes with 32 lanes of 16-byte stores.
constexpr int kOmRows = 32;

template <int NK, int JB>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(JB == 4 ? 2 : 3))) void k_gemm_outer_mfma(GemmArgs a) {
  constexpr int KS = 1 << NK;
  constexpr int kOmCols = 64 * JB, kOmRs = 32 * JB + 8;
  __shared__ float2 As[2][kOmRows * KS];
  __shared__ __align__(16) float Cs[4][kOmRows * kOmRs];
  const int64_t M = a.M, N = a.N;
  const int64_t col_blocks = N / kOmCols;
  const int64_t row_blocks = int64_t(gridDim.x) / col_blocks;
  const int64_t mrows = (M + row_blocks - 1) / row_blocks;
  const int64_t cb = int64_t(blockIdx.x) % col_blocks, mb = int64_t(blockIdx.x) / col_blocks;
  const int64_t n0 = cb * kOmCols, mw0 = mb * mrows;
  const int64_t z = int64_t(blockIdx.y) + int64_t(blockIdx.z) * gridDim.y;
  if (z >= a.rows * a.nb) return;
  const int64_t sl = z / a.rows, r = z - sl * a.rows;
  const int64_t ar = a.ga ? a.ga[r] : (a.a_rows == 1 ? 0 : r);
  const int64_t br = a.gb ? a.gb[r] : (a.b_rows == 1 ? 0 : r);
  const float2* A = a.A + sl * a.a_slice_stride + ar * a.a_row_stride;
  const float2* B = a.B + sl * a.b_slice_stride + br * a.b_row_stride;
  float* C = reinterpret_cast<float*>(a.C + sl * a.c_slice_stride + r * a.c_row_stride);
  float sa = 1.f, sb = 1.f;
  if (a.rec_c) {
    int sha, shb, ea, eb;
    rec_load(a.rec_a, a.rec_a_step, sl, false, sha, ea);
    rec_load(a.rec_b, a.rec_b_step, sl, false, shb, eb);
    sa = pow2f(sha);
    sb = pow2f(shb);
    if (blockIdx.x == 0 && r == 0 && threadIdx.x == 0)
      a.rec_c[sl * a.rec_c_step + kRecExp] = uint32_t(ea + eb - sha - shb);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int half = lane >> 5, j32 = lane & 31;
  // B fragments: real k row `half` of the embedding, real column j32 of block j
  float bf[JB][KS];
#pragma unroll
  for (int j = 0; j < JB; ++j) {
    const int64_t n = n0 + wave * 16 * JB + j * 16 + (j32 >> 1);
    const int64_t on = scatter_u<kMaxRank>(n, a.b_npos, a.nn);
    const bool take_im = (half != (j32 & 1));
    const float sign = (half == 1 && (j32 & 1) == 0) ? -sb : sb;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const float2 v = B[on + scatter_u<NK>(k, a.b_kpos, NK)];
      bf[j][k] = (take_im ? v.y : v.x) * sign;
    }
  }
  const int64_t mloc_mask = (int64_t(1) << a.nm) - 1;
  const int64_t m_end = (mw0 + mrows < M) ? mw0 + mrows : M;
  // staging: 32 rows x KS values of A, zero past m_end
  auto stage = [&](int buf, int64_t m0) {
    for (int e = threadIdx.x; e < kOmRows * KS; e += kThreads) {
      const int i = e / KS, k = e % KS;
      const int64_t m = m0 + i;
      float2 v = make_float2(0.f, 0.f);
      if (m < m_end) {
        const int64_t mo = (a.fold ? (m >> a.nm) * a.fold_stride : 0) +
                           scatter_u<kMaxRank>(m & mloc_mask, a.a_mpos, a.nm);
        v = A[mo + scatter_u<NK>(k, a.a_kpos, NK)];
      }
      As[buf][e] = make_float2(v.x * sa, v.y * sa);
    }
  };
  float* patch = Cs[wave];
  float mx = 0.f;
  int buf = 0;
  stage(0, mw0);
  __syncthreads();
  for (int64_t m0 = mw0; m0 < m_end; m0 += kOmRows) {
    if (m0 + kOmRows < m_end) stage(buf ^ 1, m0 + kOmRows);   // read after the next barrier
    f32x16 acc[JB];
#pragma unroll
    for (int j = 0; j < JB; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[j][v] = 0.f;
    const float2* as = As[buf] + j32 * KS;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const float2 av = as[k];
      const float af = half ? av.y : av.x;
#pragma unroll
      for (int j = 0; j < JB; ++j)
        acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af, bf[j][k], acc[j], 0, 0, 0);
    }
    // accumulators -> this wave's patch (row 8 (v/4) + 4 half + v%4, real column 32 j + j32)
#pragma unroll
    for (int j = 0; j < JB; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        mx = fmaxf(mx, fabsf(acc[j][v]));   // rows past m_end hold exact zeros
        patch[(8 * (v >> 2) + 4 * half + (v & 3)) * kOmRs + 32 * j + j32] = acc[j][v];
      }
    // the patch is this wave's alone: its LDS operations complete in order
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // 16 bytes per lane, 8 JB lanes per row: each row's 128 JB contiguous bytes in one piece
    constexpr int LPR = 8 * JB, RPI = 64 / LPR;   // lanes per row, rows per instruction
    const int rows_left = int(m_end - m0 < kOmRows ? m_end - m0 : kOmRows);
    const int rl = lane / LPR, cl = lane % LPR;
    float* cm = C + m0 * N * 2 + (n0 + wave * 16 * JB) * 2 + 4 * cl;
#pragma unroll
    for (int t = 0; t < kOmRows / RPI; ++t) {
      const int row = RPI * t + rl;
      const float4 x = *reinterpret_cast<const float4*>(&patch[row * kOmRs + 4 * cl]);
      if (row < rows_left) *reinterpret_cast<float4*>(cm + row * int(N) * 2) = x;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __syncthreads();   // the staged rows have been read and the next ones written
    buf ^= 1;
  }
  if (a.rec_c) amax_commit_wg(mx, sl, a.rec_c, a.rec_c_step);
}

// ---------------------------------------------------------------------------------
// split-precision complex GEMM: every FP32 operand value x is split while it is staged
// into LDS as hi = bf16(x), lo = bf16(x - hi); the product is hi*hi + hi*lo + lo*hi with
// FP32 accumulation (the lo*lo term, ~2^-16 relative, is dropped).  A is kept as the real
// M x 2K matrix of its interleaved parts; B is written in LDS directly in its real
// embedding, transposed so that one lane's eight consecutive K values are contiguous:
//   column 2n   (real part of C):      (Re B, -Im B) for every complex k
//   column 2n+1 (imaginary part of C): (Im B,  Re B)
// One v_mfma_f32_32x32x16_bf16 then consumes 8 complex k for 32 rows x 16 complex columns.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));



typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// (re, im) * scale -> packed FP16 words hi = fp16(x), lo = fp16(x - hi) (x = scaled value,
// round to nearest even); the power-of-two scale keeps |x| below 2^14
__device__ __forceinline__ void split_pair_f16(float2 v, float scale, uint32_t& hi, uint32_t& lo) {
  f32x2v x;
  x[0] = v.x * scale;
  x[1] = v.y * scale;
  const f16x2 h = __builtin_convertvector(x, f16x2);
  hi = __builtin_bit_cast(uint32_t, h);
  const f32x2v r = x - __builtin_convertvector(h, f32x2v);
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, f16x2));
}

// (re, im) -> packed bf16 words hi = (bf16(re), bf16(im)), lo = (bf16(re - hi.re),
// bf16(im - hi.im)), low half first; conversions round to nearest even
__device__ __forceinline__ void split_pair(float2 x, uint32_t& hi, uint32_t& lo) {
  f32x2v v;
  v[0] = x.x;
  v[1] = x.y;
  const bf16x2 h = __builtin_convertvector(v, bf16x2);
  hi = __builtin_bit_cast(uint32_t, h);
  f32x2v r;
  r[0] = x.x - __builtin_bit_cast(float, hi << 16);
  r[1] = x.y - __builtin_bit_cast(float, hi & 0xffff0000u);
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, bf16x2));
}

// MODE 0: BF16 split while staging; 2: FP16 split of operands scaled by a power of two
// per slice that brings their largest component to [2^13, 2^14) (scale records: the output
// keeps the product of the two scales, recorded in its exponent)
template <int WAVES_M, int WAVES_N, int UM, int UN, bool A_MFAST, bool B_NFAST, int MODE>
__global__ __launch_bounds__(WAVES_M * WAVES_N * 64) void k_gemm_bf16x3(GemmArgs a) {
  constexpr bool F16 = (MODE == 2);
  constexpr int NT = WAVES_M * WAVES_N * 64;   // four or eight waves
  static_assert(NT == 256 || NT == 512, "four or eight waves per workgroup");
  constexpr int BK = 16;                       // complex k per LDS stage (two MFMA steps)
  constexpr int BM = WAVES_M * UM * 32;
  constexpr int BN = WAVES_N * UN * 16;
  using Tile = GemmTile<BM, BN, BK, A_MFAST, B_NFAST, false, NT>;
  constexpr int A_LD = Tile::A_LD, B_LD = Tile::B_LD;
  constexpr int RS = 2 * BK;                   // bf16 per LDS row (32 real k, 64 bytes)
  constexpr int A_PLANE = BM * RS, B_PLANE = 2 * BN * RS;
  // chunk rotation of row r: c ^ ((r >> 1) ^ (r >> S2) ^ (r >> S3)), shifts per tile width
  constexpr int LBN = BN >= 128 ? 7 : BN >= 64 ? 6 : BN >= 32 ? 5 : 4;
  constexpr int S2 = BN <= 16 ? 3 : 2, S3 = BN <= 16 ? 4 : LBN - 1;
  constexpr int STAGE = 2 * A_PLANE + 2 * B_PLANE;   // hi and lo planes of A and B
  __shared__ __attribute__((aligned(16))) __bf16 lds[2 * STAGE];

  Tile t;
  if (!t.init(a)) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave % WAVES_M, wn = wave / WAVES_M;
  // operand scales from the scale records: FP16 always (hi below 2^14, far from FP16's
  // limit), BF16 (FP32's exponent range) only for operands far from 1
  float sc_a = 1.f, sc_b = 1.f;
  if (a.rec_c) rec_scales(a, t.sl, F16, t.first_of_slice(), sc_a, sc_b);

  f32x16 acc[UM][UN];
#pragma unroll
  for (int i = 0; i < UM; ++i)
#pragma unroll
    for (int j = 0; j < UN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  float2 ra[A_LD], rb[B_LD];
  uint32_t valid = 0;
  // LDS rows hold 32 bf16 of k in four 16-byte chunks, unpadded; chunk c of row r is stored
  // at position c ^ ((r >> 1) ^ (r >> S2) ^ (r >> S3)) & 3.  The embedded B column 2n + c
  // (c = 0: (re, -im), c = 1: (im, re)) is LDS row n + BN c.  With this layout the 16-byte
  // staging writes and fragment reads of the tile shapes in use are free of bank conflicts
  // on a 64-bank LDS (16 lanes per 16-byte access) and nearly so on a 32-bank one.
  auto lds_off = [](int row, int kq) {
    const int rot = (row >> 1) ^ (row >> S2) ^ (row >> S3);
    return row * RS + ((((kq >> 3) ^ rot) & 3) << 3) + (kq & 7);
  };
  // LDS element offsets of this thread's load slots (A: row-major k pairs; B: the two
  // embedded columns 2n and 2n + 1 of its (k, n) value, LDS rows n and BN + n)
  int a_so[A_LD], b_so0[B_LD], b_so1[B_LD];
#pragma unroll
  for (int i = 0; i < A_LD; ++i) a_so[i] = lds_off(Tile::a_row(i), 2 * Tile::a_col(i));
#pragma unroll
  for (int i = 0; i < B_LD; ++i) {
    b_so0[i] = lds_off(Tile::b_n(i), 2 * Tile::b_kr(i));
    b_so1[i] = lds_off(BN + Tile::b_n(i), 2 * Tile::b_kr(i));
  }
  auto store = [&](int stage) {
    if (valid != t.full_bits) Tile::apply(valid, ra, rb);
    __bf16* ah = lds + stage * STAGE;
    __bf16* al = ah + A_PLANE;
    __bf16* bh = al + A_PLANE;
    __bf16* bl = bh + B_PLANE;
    uint32_t wh[A_LD + B_LD], wl[A_LD + B_LD];   // packed (re, im) hi and lo words
    if (F16) {
#pragma unroll
      for (int i = 0; i < A_LD; ++i) split_pair_f16(ra[i], sc_a, wh[i], wl[i]);
#pragma unroll
      for (int i = 0; i < B_LD; ++i) split_pair_f16(rb[i], sc_b, wh[A_LD + i], wl[A_LD + i]);
    } else {
      if (sc_a != 1.f || sc_b != 1.f) Tile::scale(sc_a, sc_b, ra, rb);
#pragma unroll
      for (int i = 0; i < A_LD + B_LD; ++i) split_pair(i < A_LD ? ra[i] : rb[i - A_LD], wh[i], wl[i]);
    }
    if (A_MFAST) {
      // a thread's A slots are consecutive k of one row: whole 16-byte chunks
#pragma unroll
      for (int c = 0; c < A_LD / 4; ++c) {
        *reinterpret_cast<uint4*>(&ah[a_so[4 * c]]) =
            make_uint4(wh[4 * c], wh[4 * c + 1], wh[4 * c + 2], wh[4 * c + 3]);
        *reinterpret_cast<uint4*>(&al[a_so[4 * c]]) =
            make_uint4(wl[4 * c], wl[4 * c + 1], wl[4 * c + 2], wl[4 * c + 3]);
      }
    } else {
#pragma unroll
      for (int i = 0; i < A_LD; ++i) {
        *reinterpret_cast<uint32_t*>(&ah[a_so[i]]) = wh[i];
        *reinterpret_cast<uint32_t*>(&al[a_so[i]]) = wl[i];
      }
    }
    // embedded B: column 2n holds (re, -im) = the hi/lo word with the upper half's sign
    // flipped, column 2n+1 holds (im, re) = the halves swapped
    auto col0 = [](uint32_t w) { return w ^ 0x80000000u; };
    auto col1 = [](uint32_t w) { return (w >> 16) | (w << 16); };
    if (B_NFAST && B_LD % 4 == 0) {
      // a thread's B slots are consecutive k of one column: whole 16-byte chunks
#pragma unroll
      for (int c = 0; c < B_LD / 4; ++c) {
        const uint32_t* h = wh + A_LD + 4 * c;
        const uint32_t* l = wl + A_LD + 4 * c;
        *reinterpret_cast<uint4*>(&bh[b_so0[4 * c]]) = make_uint4(col0(h[0]), col0(h[1]), col0(h[2]), col0(h[3]));
        *reinterpret_cast<uint4*>(&bh[b_so1[4 * c]]) = make_uint4(col1(h[0]), col1(h[1]), col1(h[2]), col1(h[3]));
        *reinterpret_cast<uint4*>(&bl[b_so0[4 * c]]) = make_uint4(col0(l[0]), col0(l[1]), col0(l[2]), col0(l[3]));
        *reinterpret_cast<uint4*>(&bl[b_so1[4 * c]]) = make_uint4(col1(l[0]), col1(l[1]), col1(l[2]), col1(l[3]));
      }
    } else {
#pragma unroll
      for (int i = 0; i < B_LD; ++i) {
        if (!Tile::b_slot(i)) continue;
        const uint32_t h = wh[A_LD + i], l = wl[A_LD + i];
        *reinterpret_cast<uint32_t*>(&bh[b_so0[i]]) = col0(h);
        *reinterpret_cast<uint32_t*>(&bh[b_so1[i]]) = col1(h);
        *reinterpret_cast<uint32_t*>(&bl[b_so0[i]]) = col0(l);
        *reinterpret_cast<uint32_t*>(&bl[b_so1[i]]) = col1(l);
      }
    }
  };

  const int half = lane >> 5, j32 = lane & 31;
  int a_rd[2][UM], b_rd[2][UN];   // per k step: 16 bytes at k = 8 (half + 2 step)
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
#pragma unroll
    for (int i = 0; i < UM; ++i) a_rd[ks][i] = lds_off(wm * UM * 32 + i * 32 + j32, 8 * (half + 2 * ks));
#pragma unroll
    for (int j = 0; j < UN; ++j)
      b_rd[ks][j] = lds_off(wn * UN * 16 + j * 16 + (j32 >> 1) + BN * (j32 & 1), 8 * (half + 2 * ks));
  }

  int stage = 0;
  if (t.k_begin < t.k_end) {
    t.load(a, t.k_begin, ra, rb, valid);
    store(0);
  }
  __syncthreads();
  for (int64_t k0 = t.k_begin; k0 < t.k_end; k0 += BK) {
    const bool more = k0 + BK < t.k_end;
    if (more) t.load(a, k0 + BK, ra, rb, valid);
    const __bf16* ah = lds + stage * STAGE;
    const __bf16* al = ah + A_PLANE;
    const __bf16* bh = al + A_PLANE;
    const __bf16* bl = bh + B_PLANE;
#pragma unroll
    for (int kstep = 0; kstep < 2; ++kstep) {
      // B fragments for the whole step, A fragments one tile row at a time (fewer live
      // registers for the 4 x 4 tiles of the large configuration)
      bf16x8 xbh[UN], xbl[UN];
#pragma unroll
      for (int j = 0; j < UN; ++j) {
        xbh[j] = *reinterpret_cast<const bf16x8*>(&bh[b_rd[kstep][j]]);
        xbl[j] = *reinterpret_cast<const bf16x8*>(&bl[b_rd[kstep][j]]);
      }
#pragma unroll
      for (int i = 0; i < UM; ++i) {
        const bf16x8 xah = *reinterpret_cast<const bf16x8*>(&ah[a_rd[kstep][i]]);
        const bf16x8 xal = *reinterpret_cast<const bf16x8*>(&al[a_rd[kstep][i]]);
#pragma unroll
        for (int j = 0; j < UN; ++j) {
          if constexpr (F16) {
            const f16x8 ah8 = __builtin_bit_cast(f16x8, xah), al8 = __builtin_bit_cast(f16x8, xal);
            const f16x8 bh8 = __builtin_bit_cast(f16x8, xbh[j]), bl8 = __builtin_bit_cast(f16x8, xbl[j]);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al8, bh8, acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah8, bl8, acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah8, bh8, acc[i][j], 0, 0, 0);
          } else {
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xal, xbh[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xah, xbl[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xah, xbh[j], acc[i][j], 0, 0, 0);
          }
        }
      }
    }
    if (more) store(stage ^ 1);
    __syncthreads();
    stage ^= 1;
  }
  if (a.rec_c && a.k_splits == 1)
    amax_commit_wg(Tile::template acc_absmax<UM, UN>(acc), t.sl, a.rec_c, a.rec_c_step);
  t.template store_acc<UM, UN>(a, acc, wm * UM * 32, wn * UN * 16);
}

__global__ __launch_bounds__(kThreads) void k_zero_u32(uint32_t* p, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kThreads)
    p[i] = 0u;
}

__global__ __launch_bounds__(kThreads) void k_reduce(ReduceArgs a) {
  if (a.rec) {
    // wave-uniform trip count, so that every lane takes part in amax_commit
    for (int64_t b = int64_t(blockIdx.x) * kThreads + (threadIdx.x & ~63); b < a.elems;
         b += int64_t(gridDim.x) * kThreads) {
      const int64_t i = b + (threadIdx.x & 63);
      float m = 0.f;
      int64_t slice = -1;
      if (i < a.elems) {
        float2 s = a.partial[i];
        for (int k = 1; k < a.splits; ++k) {
          const float2 p = a.partial[int64_t(k) * a.elems + i];
          s.x += p.x;
          s.y += p.y;
        }
        a.C[i] = s;
        m = fmaxf(fabsf(s.x), fabsf(s.y));
        slice = i / a.slice_elems;
      }
      amax_commit(m, slice, a.rec, a.rec_step);
    }
    return;
  }
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < a.elems;
       i += int64_t(gridDim.x) * kThreads) {
    float2 s = a.partial[i];
    for (int k = 1; k < a.splits; ++k) {
      const float2 p = a.partial[int64_t(k) * a.elems + i];
      s.x += p.x;
      s.y += p.y;
    }
    a.C[i] = s;
  }
}

// Many splits: 64 elements per workgroup, each wave sums a quarter of the splits (two
// interleaved chains), and the four partial sums are added in wave order.  The summation
// order is fixed by the split count alone.
__global__ __launch_bounds__(kThreads) void k_reduce_wide(ReduceArgs a) {
  __shared__ float2 red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = int64_t(blockIdx.x) * 64 + lane;
  const int per = (a.splits + 3) / 4;
  const int s0 = w * per, s1 = (s0 + per < a.splits) ? s0 + per : a.splits;
  float2 c0 = make_float2(0.f, 0.f), c1 = make_float2(0.f, 0.f);
  if (i < a.elems) {
    int k = s0;
    for (; k + 1 < s1; k += 2) {
      const float2 p0 = a.partial[int64_t(k) * a.elems + i];
      const float2 p1 = a.partial[int64_t(k + 1) * a.elems + i];
      c0.x += p0.x;
      c0.y += p0.y;
      c1.x += p1.x;
      c1.y += p1.y;
    }
    if (k < s1) {
      const float2 p0 = a.partial[int64_t(k) * a.elems + i];
      c0.x += p0.x;
      c0.y += p0.y;
    }
  }
  red[w][lane] = make_float2(c0.x + c1.x, c0.y + c1.y);
  __syncthreads();
  if (w == 0) {
    float m = 0.f;
    int64_t slice = -1;
    if (i < a.elems) {
      float2 t = red[0][lane];
#pragma unroll
      for (int q = 1; q < 4; ++q) {
        t.x += red[q][lane].x;
        t.y += red[q][lane].y;
      }
      a.C[i] = t;
      m = fmaxf(fabsf(t.x), fabsf(t.y));
      slice = i / a.slice_elems;
    }
    if (a.rec) amax_commit(m, slice, a.rec, a.rec_step);
  }
}

// ---------------------------------------------------------------------------------
// slices
__global__ __launch_bounds__(kThreads) void k_slice_leaves(SliceLeafArgs a, int64_t per_slice) {
  const int64_t base = *a.base;
  const int64_t total = per_slice * a.nb;
  for (int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x; g < total;
       g += int64_t(gridDim.x) * kThreads) {
    const int64_t sl = g / per_slice, gg = g - sl * per_slice;
    const uint64_t* sigma = a.slice_ids + 2 * (base + sl);   // two words per id
    int e = 0;
    while (e + 1 < a.n_entries && a.prefix[e + 1] <= gg) ++e;
    const SliceLeafEntry& t = a.table[e];
    const int64_t o = gg - a.prefix[e];
    const int64_t row = o >> t.dense_out;
    int64_t d = o & ((int64_t(1) << t.dense_out) - 1);
    for (int j = 0; j < t.n_sl; ++j) {
      const int p = t.pos[j];
      const int b = t.bit[j];
      const int64_t v = (sigma[b >> 6] >> (b & 63)) & 1;
      d = ((d >> p) << (p + 1)) | (v << p) | (d & ((int64_t(1) << p) - 1));
    }
    const int64_t src = t.src_off + (row << (t.dense_out + t.n_sl)) + d;
    a.ws[t.dst_off + sl * t.elems_out + o] = a.consts[src];
  }
}

__global__ __launch_bounds__(kThreads) void k_slice_sum(SliceSumArgs a) {
  const int64_t l = int64_t(1) << a.n_open;
  const int64_t total = a.L * l;
  for (int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x; g < total;
       g += int64_t(gridDim.x) * kThreads) {
    const int64_t grp = g >> a.n_open, mu = g & (l - 1);
    int64_t off = int64_t(a.row_of[grp]) * a.f_row_stride;
    for (int t = 0; t < a.n_open; ++t)
      if ((mu >> (a.n_open - 1 - t)) & 1) off += a.open_stride[t];
    double2* out = reinterpret_cast<double2*>(a.amps) + g;
    double2 o = a.overwrite ? make_double2(0.0, 0.0) : *out;
    for (int64_t sl = 0; sl < a.nb; ++sl) {     // slice order, one rounding per slice
      const float2 v = a.F[sl * a.f_slice_stride + off];
      // the stored values times 2^E (exact in FP64)
      const double f = a.rec_f ? ldexp(1.0, int(a.rec_f[sl * a.rec_f_step + kRecExp])) : 1.0;
      o.x += double(v.x) * f;
      o.y += double(v.y) * f;
    }
    *out = o;
  }
}

__global__ void k_set_i64(int64_t* p, int64_t v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *p = v;
}

__global__ void k_add_i64(int64_t* p, int64_t v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *p += v;
}

__global__ __launch_bounds__(kThreads) void k_fill_zero(double* p, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kThreads)
    p[i] = 0.0;
}

// ---------------------------------------------------------------------------------
// norm: partial sums in a fixed order, then one block folds them
__global__ __launch_bounds__(kThreads) void k_norm_partial(const double* amps, int64_t n,
                                                           double* partials) {
  __shared__ double red[kThreads];
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kThreads) {
    const double re = amps[2 * i], im = amps[2 * i + 1];
    s += re * re + im * im;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kThreads) void k_norm_final(const double* partials, int n,
                                                         double* out) {
  __shared__ double red[kThreads];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) s += partials[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// ---------------------------------------------------------------------------------
// sampling: SplitMix64 (Steele, Lea & Flood 2014) as a counter-based generator
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t j) {
  uint64_t z = seed + (j + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double weight(const double* amps, int64_t i) {
  // re^2 + im^2 rounded step by step (no fused multiply-add), as a sequential host
  // computation would round it
  return __dadd_rn(__dmul_rn(amps[2 * i], amps[2 * i]), __dmul_rn(amps[2 * i + 1], amps[2 * i + 1]));
}

__device__ __forceinline__ uint64_t compose(uint64_t closed, int64_t mu, int n_open,
                                            const int32_t* open_q, int n) {
  uint64_t x = closed;
  for (int t = 0; t < n_open; ++t)
    if ((mu >> (n_open - 1 - t)) & 1) x |= uint64_t(1) << (n - 1 - open_q[t]);
  return x;
}

__global__ void k_cumsum_one_group(const double* amps, int64_t l, double* cum) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double c = 0.0;
  for (int64_t i = 0; i < l; ++i) {
    c = __dadd_rn(c, weight(amps, i));
    cum[i] = c;
  }
}

__global__ __launch_bounds__(kThreads) void k_sample_one_group(
    const double* cum, int64_t l, uint64_t closed, int n_open, const int32_t* open_q, int n,
    uint64_t seed, int64_t n_samples, uint64_t* out) {
  for (int64_t j = int64_t(blockIdx.x) * kThreads + threadIdx.x; j < n_samples;
       j += int64_t(gridDim.x) * kThreads) {
    const double u = double(splitmix64(seed, uint64_t(j)) >> 11) * 0x1.0p-53;
    const double total = cum[l - 1];
    int64_t mu;
    if (total == 0.0) {
      mu = int64_t(u * double(l));
      if (mu > l - 1) mu = l - 1;
    } else {
      const double target = __dmul_rn(u, total);
      int64_t lo = 0, hi = l - 1;     // smallest mu with cum[mu] > target
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cum[mid] > target) hi = mid; else lo = mid + 1;
      }
      mu = lo;
    }
    out[j] = compose(closed, mu, n_open, open_q, n);
  }
}

__global__ __launch_bounds__(kThreads) void k_sample_groups(
    const double* amps, int64_t L, int n_open, const uint64_t* closed, const int32_t* open_q,
    int n, uint64_t seed, uint64_t* out) {
  const int64_t l = int64_t(1) << n_open;
  for (int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x; g < L;
       g += int64_t(gridDim.x) * kThreads) {
    const double* a = amps + 2 * g * l;
    double total = 0.0;
    for (int64_t i = 0; i < l; ++i) total = __dadd_rn(total, weight(a, i));
    const double u = double(splitmix64(seed, uint64_t(g)) >> 11) * 0x1.0p-53;
    int64_t mu = l - 1;
    if (total == 0.0) {
      mu = int64_t(u * double(l));
      if (mu > l - 1) mu = l - 1;
    } else {
      const double target = __dmul_rn(u, total);
      double c = 0.0;
      for (int64_t i = 0; i < l; ++i) {
        c = __dadd_rn(c, weight(a, i));
        if (c > target) { mu = i; break; }
      }
    }
    out[g] = compose(closed[g], mu, n_open, open_q, n);
  }
}

__device__ __forceinline__ double unif(uint64_t seed, uint64_t k) {
  return double(splitmix64(seed, k) >> 11) * 0x1.0p-53;
}

__device__ __forceinline__ int64_t index_of(double u, int64_t l) {
  const int64_t i = int64_t(__dmul_rn(u, double(l)));
  return i < l - 1 ? i : l - 1;
}

// In-group Metropolis chains, one thread per draw d (draws d0 + 0..n-1; group d for several
// groups, else group 0): start floor(u_k0 l), k0 = d (2 steps + 1); step t proposes
// floor(u_(k0+2t-1) l) and moves iff w_nu >= u_(k0+2t) w_mu.
__global__ __launch_bounds__(kThreads) void k_sample_metropolis(
    const double* amps, int64_t L, int n_open, const uint64_t* closed, const int32_t* open_q,
    int n, uint64_t seed, int64_t d0, int64_t n_draws, int steps, uint64_t* out) {
  const int64_t l = int64_t(1) << n_open;
  for (int64_t j = int64_t(blockIdx.x) * kThreads + threadIdx.x; j < n_draws;
       j += int64_t(gridDim.x) * kThreads) {
    const int64_t d = d0 + j, g = L > 1 ? d : 0;
    const double* a = amps + 2 * g * l;
    const uint64_t k0 = uint64_t(d) * uint64_t(2 * steps + 1);
    int64_t mu = index_of(unif(seed, k0), l);
    double wmu = weight(a, mu);
    for (int t = 1; t <= steps; ++t) {
      const int64_t nu = index_of(unif(seed, k0 + 2 * t - 1), l);
      const double wnu = weight(a, nu);
      if (wnu >= __dmul_rn(unif(seed, k0 + 2 * t), wmu)) {
        mu = nu;
        wmu = wnu;
      }
    }
    out[j] = compose(closed[g], mu, n_open, open_q, n);
  }
}

// Frugal rejection sampling, one thread per draw: k0 = 2 d trials; proposal t is
// floor(u_(k0+2t) l), accepted iff u_(k0+2t+1) (m S) < w_nu l with S the group's weight sum
// in mu order (totals[g]); after `trials` rejections the last proposal is kept.
__global__ __launch_bounds__(kThreads) void k_sample_frugal(
    const double* amps, const double* totals, int64_t L, int n_open, const uint64_t* closed,
    const int32_t* open_q, int n, uint64_t seed, int64_t d0, int64_t n_draws, double m,
    int trials, uint64_t* out) {
  const int64_t l = int64_t(1) << n_open;
  for (int64_t j = int64_t(blockIdx.x) * kThreads + threadIdx.x; j < n_draws;
       j += int64_t(gridDim.x) * kThreads) {
    const int64_t d = d0 + j, g = L > 1 ? d : 0;
    const double* a = amps + 2 * g * l;
    const double ms = __dmul_rn(m, totals[g]);
    const uint64_t k0 = uint64_t(d) * uint64_t(2 * trials);
    int64_t nu = 0;
    for (int t = 0; t < trials; ++t) {
      nu = index_of(unif(seed, k0 + 2 * t), l);
      if (__dmul_rn(unif(seed, k0 + 2 * t + 1), ms) < __dmul_rn(weight(a, nu), double(l))) break;
    }
    out[j] = compose(closed[g], nu, n_open, open_q, n);
  }
}

// Weight sum of each group in mu order (one thread per group).
__global__ __launch_bounds__(kThreads) void k_group_totals(const double* amps, int64_t L,
                                                           int64_t l, double* totals) {
  for (int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x; g < L;
       g += int64_t(gridDim.x) * kThreads) {
    const double* a = amps + 2 * g * l;
    double c = 0.0;
    for (int64_t i = 0; i < l; ++i) c = __dadd_rn(c, weight(a, i));
    totals[g] = c;
  }
}

int grid_for(int64_t work, int64_t per_block, int64_t cap = 8192) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return int(g);
}

template <int NK, int NN>
hipError_t launch_stream_t(const StreamArgs& a, hipStream_t s) {
  const bool s_shared = (a.s_rows == 1 && a.gs == nullptr && a.s_slice_stride == 0);
  const int64_t gy = a.nb < 65535 ? a.nb : 65535;
  const int64_t gz = (a.nb + gy - 1) / gy;
  if (s_shared) {
    const int64_t per_slice = a.rows << a.n_m;
    const int64_t cap = a.nb >= 65536 ? 1 : 65536 / a.nb;
    hipLaunchKernelGGL((k_stream<NK, NN>),
                       dim3(unsigned(grid_for(per_slice, kThreads, cap)), unsigned(gy), unsigned(gz)),
                       dim3(kThreads), 0, s, a);
    return hipGetLastError();
  }
  constexpr int KS = 1 << NK, NS = 1 << NN, E = KS * NS;
  static_assert(E <= kStageElems, "one row of the small operand must fit the stage");
  const int64_t M = int64_t(1) << a.n_m;
  int rw = 1, nsplit = 1;
  int64_t chunks;
  if (M >= kThreads) {
    chunks = a.rows * (M / kThreads);
  } else {
    const int64_t by_threads = kThreads / M, by_lds = kStageElems / E;
    rw = int(by_threads < by_lds ? by_threads : by_lds);
    const int64_t items = int64_t(rw) * M;
    const int64_t ns = kThreads / items;
    nsplit = int(ns < NS ? ns : NS);
    chunks = (a.rows + rw - 1) / rw;
  }
  hipLaunchKernelGGL((k_stream_rows<NK, NN>), dim3(unsigned(chunks), unsigned(gy), unsigned(gz)),
                     dim3(kThreads), 0, s, a, rw, nsplit);
  return hipGetLastError();
}

template <int NK>
hipError_t launch_stream_n(const StreamArgs& a, hipStream_t s) {
  switch (a.nn) {
    case 0: return launch_stream_t<NK, 0>(a, s);
    case 1: return launch_stream_t<NK, 1>(a, s);
    case 2: return launch_stream_t<NK, 2>(a, s);
    case 3: return launch_stream_t<NK, 3>(a, s);
    case 4: return launch_stream_t<NK, 4>(a, s);
  }
  return hipErrorInvalidValue;
}

template <int WM, int WN, int UM, int UN, int BK>
hipError_t launch_gemm_cfg(const GemmArgs& a, hipStream_t s) {
  constexpr int BM = WM * UM * 32, BN = WN * UN * 16;
  const int64_t tiles = ((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN);
  const int64_t zs = a.rows * a.nb * a.k_splits;
  const int64_t gy = zs < 65535 ? zs : 65535;
  const int64_t gz = (zs + gy - 1) / gy;
  const dim3 grid{unsigned(tiles), unsigned(gy), unsigned(gz)};
  const int sel = (a.a_mfast ? 1 : 0) | (a.b_nfast ? 2 : 0);
  if (a.precision == 0) {
    switch (sel) {
      case 0: hipLaunchKernelGGL((k_gemm<WM, WN, UM, UN, BK, false, false>), grid, dim3(kThreads), 0, s, a); break;
      case 1: hipLaunchKernelGGL((k_gemm<WM, WN, UM, UN, BK, true, false>), grid, dim3(kThreads), 0, s, a); break;
      case 2: hipLaunchKernelGGL((k_gemm<WM, WN, UM, UN, BK, false, true>), grid, dim3(kThreads), 0, s, a); break;
      default: hipLaunchKernelGGL((k_gemm<WM, WN, UM, UN, BK, true, true>), grid, dim3(kThreads), 0, s, a); break;
    }
  } else {
    if (a.precision != 1 && a.precision != 3) return hipErrorInvalidValue;
    const int mode = a.precision == 1 ? 0 : 2;
    switch (sel * 3 + mode) {
#define TNC_SPLIT_CASE(S, MD, AF, BF)                                                          \
  case S * 3 + MD:                                                                            \
    hipLaunchKernelGGL((k_gemm_bf16x3<WM, WN, UM, UN, AF, BF, MD>), grid, dim3(kThreads), 0, s, a); \
    break;
      TNC_SPLIT_CASE(0, 0, false, false) TNC_SPLIT_CASE(0, 2, false, false)
      TNC_SPLIT_CASE(1, 0, true, false) TNC_SPLIT_CASE(1, 2, true, false)
      TNC_SPLIT_CASE(2, 0, false, true) TNC_SPLIT_CASE(2, 2, false, true)
      TNC_SPLIT_CASE(3, 0, true, true) TNC_SPLIT_CASE(3, 2, true, true)
#undef TNC_SPLIT_CASE
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_stream(const StreamArgs& a, hipStream_t s) {
  switch (a.nk) {
    case 0: return launch_stream_n<0>(a, s);
    case 1: return launch_stream_n<1>(a, s);
    case 2: return launch_stream_n<2>(a, s);
    case 3: return launch_stream_n<3>(a, s);
    case 4: return launch_stream_n<4>(a, s);
    case 5: return launch_stream_n<5>(a, s);
    case 6: return launch_stream_n<6>(a, s);
  }
  return hipErrorInvalidValue;
}

// Tile configurations (complex elements): 0 = 128 x 64 (2x2 waves, 2x2 MFMA tiles each),
// 1 = 128 x 16 (4x1 waves, one MFMA tile each), 2 = 64 x 32 (2x2 waves, one tile each),
// 3 = 128 x 128 (2x2 waves, 2x4 MFMA tiles each), 4 = 128 x 32 (4x1 waves, 1x2 tiles each),
// 5 = 128 x 8 on 16x16x4 MFMA tiles (complex64 only; split precision uses 1), or, for rows
// of narrow long-K products, k_gemm_rows_narrow in every form.
template <int MH, int NN>
hipError_t launch_rows_narrow_t(const GemmArgs& a, hipStream_t s) {
  const int64_t waves = a.rows * a.nb, blocks = (waves + 3) / 4;
  const int64_t gx = blocks < 65535 ? blocks : 65535;
  const int64_t gy = (blocks + gx - 1) / gx;
  hipLaunchKernelGGL((k_gemm_rows_narrow<MH, NN>), dim3(unsigned(gx), unsigned(gy)), dim3(kThreads),
                     size_t(2 * a.K) * sizeof(int32_t), s, a);
  return hipGetLastError();
}

// k_gemm_rows_narrow for its shapes (see there), or an error when none applies
hipError_t launch_rows_narrow(const GemmArgs& a, hipStream_t s) {
  const int mh = int(a.M / 4);
  switch (mh * 8 + a.nn) {
    case 2 * 8 + 0: return launch_rows_narrow_t<2, 0>(a, s);
    case 2 * 8 + 1: return launch_rows_narrow_t<2, 1>(a, s);
    case 2 * 8 + 2: return launch_rows_narrow_t<2, 2>(a, s);
    case 4 * 8 + 0: return launch_rows_narrow_t<4, 0>(a, s);
    case 4 * 8 + 1: return launch_rows_narrow_t<4, 1>(a, s);
    case 4 * 8 + 2: return launch_rows_narrow_t<4, 2>(a, s);
    case 8 * 8 + 0: return launch_rows_narrow_t<8, 0>(a, s);
    case 8 * 8 + 1: return launch_rows_narrow_t<8, 1>(a, s);
    case 8 * 8 + 2: return launch_rows_narrow_t<8, 2>(a, s);
    case 16 * 8 + 0: return launch_rows_narrow_t<16, 0>(a, s);
    case 16 * 8 + 1: return launch_rows_narrow_t<16, 1>(a, s);
  }
  return hipErrorInvalidValue;
}

// Shapes k_gemm_rows_narrow takes (every form: it computes in FP32, as the short-K kernel
// does for split plans); TNC_NO_NARROW=1 turns it off.
bool gemm_rows_narrow_fits(const GemmArgs& a, bool stacked) {
  static const bool off = std::getenv("TNC_NO_NARROW") != nullptr;
  return !off && !stacked && !a.fold && a.k_splits == 1 &&
         a.M == (int64_t(1) << a.nm) && a.M >= 8 && a.M <= 64 && a.nn <= 2 &&
         a.M * a.N <= 128 && a.K >= 64 && a.K <= 4096;
}

static bool rows_narrow_fits(const GemmArgs& a) { return gemm_rows_narrow_fits(a, a.stk != nullptr); }

hipError_t launch_gemm_n8(const GemmArgs& a, hipStream_t s) {
  if (rows_narrow_fits(a)) return launch_rows_narrow(a, s);
  const int64_t tiles = ((a.M + 127) / 128) * ((a.N + 7) / 8);
  const int64_t zs = a.rows * a.nb * a.k_splits;
  const int64_t gy = zs < 65535 ? zs : 65535;
  const int64_t gz = (zs + gy - 1) / gy;
  const dim3 grid{unsigned(tiles), unsigned(gy), unsigned(gz)};
  switch ((a.a_mfast ? 1 : 0) | (a.b_nfast ? 2 : 0)) {
    case 0: hipLaunchKernelGGL((k_gemm_n8<false, false>), grid, dim3(kThreads), 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_gemm_n8<true, false>), grid, dim3(kThreads), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_gemm_n8<false, true>), grid, dim3(kThreads), 0, s, a); break;
    default: hipLaunchKernelGGL((k_gemm_n8<true, true>), grid, dim3(kThreads), 0, s, a); break;
  }
  return hipGetLastError();
}

template <int NK>
hipError_t launch_gemm_outer_k(const GemmArgs& a, hipStream_t s) {
  static const bool valu_only = std::getenv("TNC_OUTER_VALU") != nullptr;
  if constexpr (NK >= 4) {
    constexpr int JB = 4;
    if (a.N >= 64 * JB && !valu_only) {
      // rows per workgroup: up to 1024 (fewer workgroups amortise the B fragments), halved
      // while the grid would hold fewer than 512 workgroups
      const int64_t col_blocks = a.N / (64 * JB), zs = a.rows * a.nb;
      int64_t R = 1024;
      while (R > kOmRows && col_blocks * ((a.M + R - 1) / R) * zs < 512) R /= 2;
      const int64_t mrows = a.M < R ? a.M : R;
      const int64_t blocks = col_blocks * ((a.M + mrows - 1) / mrows);
      const int64_t gy = zs < 65535 ? zs : 65535;
      const int64_t gz = (zs + gy - 1) / gy;
      const dim3 grid{unsigned(blocks), unsigned(gy), unsigned(gz)};
      hipLaunchKernelGGL((k_gemm_outer_mfma<NK, JB>), grid, dim3(kThreads), 0, s, a);
      return hipGetLastError();
    }
  }
  const int64_t cols = a.N < kOuterCols ? a.N : kOuterCols;
  const int64_t mrows = a.M < kOuterRows ? a.M : kOuterRows;
  const int64_t blocks = (a.N / cols) * ((a.M + mrows - 1) / mrows);
  const int64_t zs = a.rows * a.nb;
  const int64_t gy = zs < 65535 ? zs : 65535;
  const int64_t gz = (zs + gy - 1) / gy;
  hipLaunchKernelGGL((k_gemm_outer<NK>), dim3(unsigned(blocks), unsigned(gy), unsigned(gz)),
                     dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

// The short-K kernel: K <= 16, N >= 2, M a multiple of the staged rows (or smaller), no
// row stacking and no split-K (the plan compiler only offers it then).
hipError_t launch_gemm_outer(const GemmArgs& a, hipStream_t s) {
  if (a.stk || a.k_splits != 1 || a.N < 2 || a.nk > 4) return hipErrorInvalidValue;
  switch (a.nk) {
    case 0: return launch_gemm_outer_k<0>(a, s);
    case 1: return launch_gemm_outer_k<1>(a, s);
    case 2: return launch_gemm_outer_k<2>(a, s);
    case 3: return launch_gemm_outer_k<3>(a, s);
    case 4: return launch_gemm_outer_k<4>(a, s);
  }
  return hipErrorInvalidValue;
}

// Configurations 7 and 8: eight-wave workgroups, each wave with the 2 x 2 matrix-core
// tiles of configuration 0, so one workgroup covers 128 x 128 (7) or 256 x 64 (8) complex
// outputs and every staged operand byte feeds more matrix instructions than with 128 x 64;
// split precision (96 or 80 KB of LDS per workgroup) and complex64 (k_gemm with eight
// waves, 68 or 86 KB); no row stacking.
template <int WM, int WN>
hipError_t launch_gemm_split_big_t(const GemmArgs& a, hipStream_t s) {
  constexpr int UM = 2, UN = 2;
  constexpr int BM = WM * UM * 32, BN = WN * UN * 16;
  const int64_t tiles = ((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN);
  const int64_t zs = a.rows * a.nb * a.k_splits;
  const int64_t gy = zs < 65535 ? zs : 65535;
  const int64_t gz = (zs + gy - 1) / gy;
  const dim3 grid{unsigned(tiles), unsigned(gy), unsigned(gz)};
  const int sel = (a.a_mfast ? 1 : 0) | (a.b_nfast ? 2 : 0);
  if (a.precision == 0) {      // complex64: the FP32 kernel with eight waves
    switch (sel) {
      case 0: hipLaunchKernelGGL((k_gemm<WM, WN, UM, UN, 16, false, false>), grid, dim3(WM * WN * 64), 0, s, a); break;
      case 1: hipLaunchKernelGGL((k_gemm<WM, WN, UM, UN, 16, true, false>), grid, dim3(WM * WN * 64), 0, s, a); break;
      case 2: hipLaunchKernelGGL((k_gemm<WM, WN, UM, UN, 16, false, true>), grid, dim3(WM * WN * 64), 0, s, a); break;
      default: hipLaunchKernelGGL((k_gemm<WM, WN, UM, UN, 16, true, true>), grid, dim3(WM * WN * 64), 0, s, a); break;
    }
    return hipGetLastError();
  }
  const int mode = a.precision == 1 ? 0 : 2;
  switch (sel * 3 + mode) {
#define TNC_BIG_CASE(S, MD, AF, BF)                                                            \
  case S * 3 + MD:                                                                            \
    hipLaunchKernelGGL((k_gemm_bf16x3<WM, WN, UM, UN, AF, BF, MD>), grid, dim3(WM * WN * 64), 0, s, a); \
    break;
    TNC_BIG_CASE(0, 0, false, false) TNC_BIG_CASE(0, 2, false, false)
    TNC_BIG_CASE(1, 0, true, false) TNC_BIG_CASE(1, 2, true, false)
    TNC_BIG_CASE(2, 0, false, true) TNC_BIG_CASE(2, 2, false, true)
    TNC_BIG_CASE(3, 0, true, true) TNC_BIG_CASE(3, 2, true, true)
#undef TNC_BIG_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gemm_split_big(const GemmArgs& a, hipStream_t s) {
  if (a.stk || (a.precision != 0 && a.precision != 1 && a.precision != 3)) return hipErrorInvalidValue;
  return a.config == 7 ? launch_gemm_split_big_t<2, 4>(a, s) : launch_gemm_split_big_t<4, 2>(a, s);
}

hipError_t launch_gemm(const GemmArgs& a, hipStream_t s) {
  if (a.config == 6) return launch_gemm_outer(a, s);
  if (a.config == 7 || a.config == 8) return launch_gemm_split_big(a, s);
  if (a.config == 5) {
    if (a.precision == 0 || rows_narrow_fits(a)) return launch_gemm_n8(a, s);
    GemmArgs b = a;            // the split-precision kernels have no 8-wide tile
    b.config = 1;
    return launch_gemm(b, s);
  }
  switch (a.config) {
    case 0: return launch_gemm_cfg<2, 2, 2, 2, 16>(a, s);
    case 1: return launch_gemm_cfg<4, 1, 1, 1, 16>(a, s);
    case 2: return launch_gemm_cfg<2, 2, 1, 1, 16>(a, s);
    case 3: return launch_gemm_cfg<2, 2, 2, 4, 16>(a, s);
    case 4: return launch_gemm_cfg<4, 1, 1, 2, 16>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_zero_u32(uint32_t* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s) {
  if (a.splits >= 8) {
    hipLaunchKernelGGL(k_reduce_wide, dim3(unsigned((a.elems + 63) / 64)), dim3(kThreads), 0, s, a);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_reduce, dim3(grid_for(a.elems, kThreads)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_slice_leaves(const SliceLeafArgs& a, int64_t per_slice, hipStream_t s) {
  hipLaunchKernelGGL(k_slice_leaves, dim3(grid_for(per_slice * a.nb, kThreads)), dim3(kThreads), 0,
                     s, a, per_slice);
  return hipGetLastError();
}

hipError_t launch_slice_sum(const SliceSumArgs& a, hipStream_t s) {
  const int64_t total = a.L << a.n_open;
  hipLaunchKernelGGL(k_slice_sum, dim3(grid_for(total, kThreads)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_add_i64(int64_t* p, int64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_add_i64, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_fill_zero(double* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_norm(const double* amps, int64_t n, double* partials, int n_partials,
                       double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_partial, dim3(n_partials), dim3(kThreads), 0, s, amps, n, partials);
  hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(kThreads), 0, s, partials, n_partials, out);
  return hipGetLastError();
}

hipError_t launch_sample_metropolis(const double* amps, int64_t L, int n_open, const uint64_t* closed,
                                    const int32_t* open_qubits, int n_qubits, uint64_t seed,
                                    int64_t d0, int64_t n_draws, int steps, uint64_t* out,
                                    hipStream_t s) {
  hipLaunchKernelGGL(k_sample_metropolis, dim3(grid_for(n_draws, kThreads)), dim3(kThreads), 0, s,
                     amps, L, n_open, closed, open_qubits, n_qubits, seed, d0, n_draws, steps, out);
  return hipGetLastError();
}

hipError_t launch_group_totals(const double* amps, int64_t L, int n_open, double* totals,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_group_totals, dim3(grid_for(L, kThreads)), dim3(kThreads), 0, s, amps, L,
                     int64_t(1) << n_open, totals);
  return hipGetLastError();
}

hipError_t launch_sample_frugal(const double* amps, const double* totals, int64_t L, int n_open,
                                const uint64_t* closed, const int32_t* open_qubits, int n_qubits,
                                uint64_t seed, int64_t d0, int64_t n_draws, double m, int trials,
                                uint64_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sample_frugal, dim3(grid_for(n_draws, kThreads)), dim3(kThreads), 0, s,
                     amps, totals, L, n_open, closed, open_qubits, n_qubits, seed, d0, n_draws, m,
                     trials, out);
  return hipGetLastError();
}

hipError_t launch_sample(const double* amps, int64_t L, int n_open, const uint64_t* closed,
                         const int32_t* open_q, int n, uint64_t seed, int64_t n_samples,
                         double* cum, uint64_t* out, hipStream_t s) {
  if (L == 1) {
    uint64_t c0 = 0;
    hipError_t e = hipMemcpyAsync(&c0, closed, sizeof(uint64_t), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    const int64_t l = int64_t(1) << n_open;
    hipLaunchKernelGGL(k_cumsum_one_group, dim3(1), dim3(64), 0, s, amps, l, cum);
    hipLaunchKernelGGL(k_sample_one_group, dim3(grid_for(n_samples, kThreads)), dim3(kThreads), 0, s,
                       cum, l, c0, n_open, open_q, n, seed, n_samples, out);
  } else {
    hipLaunchKernelGGL(k_sample_groups, dim3(grid_for(L, kThreads)), dim3(kThreads), 0, s, amps, L,
                       n_open, closed, open_q, n, seed, out);
  }
  return hipGetLastError();
}

}  // namespace tnc
