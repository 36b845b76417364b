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
//   k_reduce       split-K partial sums, fixed order
//   k_slice_leaves per-slice instantiation of the leaves that hold sliced bonds
//   k_slice_sum    FP64 accumulation of a slice's result into psi_hat
//   k_norm_*       FP64 sum of |amp|^2, two fixed-order passes
//   k_sample_*     inverse-CDF sampling with SplitMix64 uniforms
#include "tnc_kernels.h"

namespace tnc {

namespace {

constexpr int kThreads = 256;

// ---------------------------------------------------------------------------------
// big x small stream
template <int NK, int NN>
__global__ __launch_bounds__(kThreads) void k_stream(StreamArgs a) {
  constexpr int KS = 1 << NK, NS = 1 << NN;
  __shared__ float2 s_lds[KS * NS];
  __shared__ int64_t koff[KS];
  __shared__ int32_t soff[KS * NS];
  const bool s_shared = (a.s_rows == 1 && a.gs == nullptr && a.s_slice_stride == 0);
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
    soff[q] = so;
    if (s_shared) s_lds[q] = a.S[so];
  }
  __syncthreads();
  const int64_t per_slice = a.rows << a.n_m;
  const int64_t total = per_slice * a.nb;
  const int64_t mmask = (int64_t(1) << a.n_m) - 1;
  for (int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x; g < total;
       g += int64_t(gridDim.x) * kThreads) {
    const int64_t sl = g / per_slice, gs = g - sl * per_slice;
    const int64_t r = gs >> a.n_m, m = gs & mmask;
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
    for (int k = 0; k < KS; ++k) xv[k] = X[xo + koff[k]];
    float2 acc[NS];
#pragma unroll
    for (int n = 0; n < NS; ++n) acc[n] = make_float2(0.f, 0.f);
    if (s_shared) {
#pragma unroll
      for (int k = 0; k < KS; ++k) {
#pragma unroll
        for (int n = 0; n < NS; ++n) {
          const float2 s = s_lds[k * NS + n];
          acc[n].x += xv[k].x * s.x - xv[k].y * s.y;
          acc[n].y += xv[k].x * s.y + xv[k].y * s.x;
        }
      }
    } else {
      const int64_t sr = a.gs ? a.gs[r] : (a.s_rows == 1 ? 0 : r);
      const float2* S = a.S + sl * a.s_slice_stride + sr * a.s_row_stride;
#pragma unroll
      for (int k = 0; k < KS; ++k) {
#pragma unroll
        for (int n = 0; n < NS; ++n) {
          const float2 s = S[soff[k * NS + n]];
          acc[n].x += xv[k].x * s.x - xv[k].y * s.y;
          acc[n].y += xv[k].x * s.y + xv[k].y * s.x;
        }
      }
    }
    float2* C = a.C + sl * a.c_slice_stride + r * a.c_row_stride + (m << NN);
#pragma unroll
    for (int n = 0; n < NS; ++n) C[n] = acc[n];
  }
}

// ---------------------------------------------------------------------------------
// complex64 GEMM on v_mfma_f32_32x32x2f32
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nb) {
  // Workgroups are dealt to the 8 XCDs round-robin; renumber them so that each XCD
  // receives a contiguous range of tiles (neighbouring tiles share operand panels,
  // which then stay in that XCD's L2).
  const int64_t q = nb / 8, rem = nb % 8, x = bid % 8;
  return x * q + (x < rem ? x : rem) + bid / 8;
}

// Scatter the low `nbits` bits of x to the bit positions pos[0..nbits) (a software pdep).
__device__ __forceinline__ int64_t scatter_bits(int64_t x, const int8_t* pos, int nbits) {
  int64_t o = 0;
  for (int j = 0; j < nbits; ++j)
    if ((x >> j) & 1) o += int64_t(1) << pos[j];
  return o;
}

template <int WAVES_M, int WAVES_N, int UM, int UN, int BK, bool A_MFAST, bool B_NFAST>
__global__ __launch_bounds__(kThreads) void k_gemm(GemmArgs a) {
  static_assert(WAVES_M * WAVES_N == 4, "four waves per workgroup");
  constexpr int BM = WAVES_M * UM * 32;
  constexpr int BN = WAVES_N * UN * 16;
  constexpr int LBM = (BM == 128) ? 7 : (BM == 64 ? 6 : 5);
  constexpr int LBN = (BN == 64) ? 6 : (BN == 32 ? 5 : 4);
  constexpr int LBK = (BK == 16) ? 4 : (BK == 32 ? 5 : 3);
  constexpr int AS = 2 * BK + 2;       // floats per LDS row of A (m-major)
  constexpr int BS = 2 * BN + 2;       // floats per LDS row of B (k-major)
  constexpr int A_LD = BM * BK / kThreads;
  constexpr int B_LD = (BK * BN + kThreads - 1) / kThreads;
  __shared__ float As[BM * AS];
  __shared__ float Bs[BK * BS];

  const int64_t M = a.M, N = a.N, K = a.K;
  const int64_t tiles_m = (M + BM - 1) / BM;
  const int64_t tiles_n = (N + BN - 1) / BN;
  const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
  if (tile >= tiles_m * tiles_n) return;
  const int64_t tm = tile % tiles_m, tn = tile / tiles_m;
  const int64_t z = int64_t(blockIdx.y) + int64_t(blockIdx.z) * gridDim.y;
  const int64_t zr = z / a.k_splits;      // slice * rows + row
  const int ks = int(z % a.k_splits);
  if (zr >= a.rows * a.nb) return;
  const int64_t sl = zr / a.rows, r = zr - sl * a.rows;
  const int64_t ar = a.ga ? a.ga[r] : (a.a_rows == 1 ? 0 : r);
  const int64_t br = a.gb ? a.gb[r] : (a.b_rows == 1 ? 0 : r);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  // block bases: the tile corner's scattered offset (tile sizes divide the group sizes
  // whenever the group is larger than the tile, so corner and in-tile bits are disjoint)
  const int64_t mloc_mask = (int64_t(1) << a.nm) - 1;
  const float2* __restrict__ A = a.A + sl * a.a_slice_stride + ar * a.a_row_stride +
                                (a.fold ? (m0 >> a.nm) * a.fold_stride : 0) +
                                scatter_bits(m0 & mloc_mask, a.a_mpos, a.nm);
  const float2* __restrict__ B =
      a.B + sl * a.b_slice_stride + br * a.b_row_stride + scatter_bits(n0, a.b_npos, a.nn);
  const int64_t k_begin = int64_t(ks) * a.k_chunk;
  const int64_t k_end = (k_begin + a.k_chunk < K) ? k_begin + a.k_chunk : K;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave % WAVES_M, wn = wave / WAVES_M;

  // per-thread load slots: fixed (row, col) inside the tile, fixed scattered offsets
  int64_t a_off[A_LD], b_off[B_LD];
  bool a_in[A_LD], b_in[B_LD];
  const int nbm = a.nm < LBM ? a.nm : LBM, nbk = a.nk < LBK ? a.nk : LBK;
  const int nbn = a.nn < LBN ? a.nn : LBN;
#pragma unroll
  for (int i = 0; i < A_LD; ++i) {
    const int q = threadIdx.x + i * kThreads;
    int row, col;
    if (A_MFAST) { row = q % BM; col = q / BM; } else { row = q / BK; col = q % BK; }
    a_off[i] = scatter_bits(row, a.a_mpos, nbm) + scatter_bits(col, a.a_kpos, nbk);
    a_in[i] = (m0 + row < M);
  }
#pragma unroll
  for (int i = 0; i < B_LD; ++i) {
    const int q = threadIdx.x + i * kThreads;
    int kr, n;
    if (B_NFAST) { kr = q / BN; n = q % BN; } else { n = q / BK; kr = q % BK; }
    b_off[i] = scatter_bits(kr, a.b_kpos, nbk) + scatter_bits(n, a.b_npos, nbn);
    b_in[i] = (q < BK * BN) && (n0 + n < N);
  }

  f32x16 acc[UM][UN];
#pragma unroll
  for (int i = 0; i < UM; ++i)
#pragma unroll
    for (int j = 0; j < UN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  float2 ra[A_LD], rb[B_LD];
  auto load = [&](int64_t k0) {
    const int64_t ka = scatter_bits(k0, a.a_kpos, a.nk);
    const int64_t kb = scatter_bits(k0, a.b_kpos, a.nk);
#pragma unroll
    for (int i = 0; i < A_LD; ++i) {
      const int q = threadIdx.x + i * kThreads;
      const int col = A_MFAST ? q / BM : q % BK;
      float2 v = make_float2(0.f, 0.f);
      if (a_in[i] && k0 + col < k_end) v = A[ka + a_off[i]];
      ra[i] = v;
    }
#pragma unroll
    for (int i = 0; i < B_LD; ++i) {
      const int q = threadIdx.x + i * kThreads;
      const int kr = B_NFAST ? q / BN : q % BK;
      float2 v = make_float2(0.f, 0.f);
      if (b_in[i] && k0 + kr < k_end) v = B[kb + b_off[i]];
      rb[i] = v;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < A_LD; ++i) {
      const int q = threadIdx.x + i * kThreads;
      int row, col;
      if (A_MFAST) { row = q % BM; col = q / BM; } else { row = q / BK; col = q % BK; }
      *reinterpret_cast<float2*>(&As[row * AS + 2 * col]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < B_LD; ++i) {
      const int q = threadIdx.x + i * kThreads;
      if (q >= BK * BN) continue;
      int kr, n;
      if (B_NFAST) { kr = q / BN; n = q % BN; } else { n = q / BK; kr = q % BK; }
      *reinterpret_cast<float2*>(&Bs[kr * BS + 2 * n]) = rb[i];
    }
  };

  const int half = lane >> 5;          // 0: lanes carry Re(A); 1: lanes carry Im(A)
  const int j32 = lane & 31;
  const int bc = j32 & 1;              // output column parity: 0 = real part, 1 = imaginary
  if (k_begin < k_end) load(k_begin);
  for (int64_t k0 = k_begin; k0 < k_end; k0 += BK) {
    __syncthreads();
    store();
    __syncthreads();
    if (k0 + BK < k_end) load(k0 + BK);
#pragma unroll 4
    for (int kk = 0; kk < BK; ++kk) {
      float af[UM], bf[UN];
#pragma unroll
      for (int i = 0; i < UM; ++i)
        af[i] = As[(wm * UM * 32 + i * 32 + j32) * AS + 2 * kk + half];
#pragma unroll
      for (int j = 0; j < UN; ++j) {
        const int np = wn * UN * 16 + j * 16 + (j32 >> 1);
        const float2 b = *reinterpret_cast<const float2*>(&Bs[kk * BS + 2 * np]);
        // real embedding of B: rows (Re k, Im k) x columns (Re n, Im n)
        bf[j] = half == 0 ? (bc == 0 ? b.x : b.y) : (bc == 0 ? -b.y : b.x);
      }
#pragma unroll
      for (int i = 0; i < UM; ++i)
#pragma unroll
        for (int j = 0; j < UN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  }

  float* out = (a.k_splits > 1)
                   ? reinterpret_cast<float*>(a.partial + (int64_t(ks) * a.rows * a.nb + zr) * M * N)
                   : reinterpret_cast<float*>(a.C + sl * a.c_slice_stride + r * a.c_row_stride);
#pragma unroll
  for (int i = 0; i < UM; ++i)
#pragma unroll
    for (int j = 0; j < UN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        // 32x32 accumulator layout: column = lane % 32, row = 8 (v/4) + 4 (lane/32) + v%4
        const int row = wm * UM * 32 + i * 32 + 8 * (v >> 2) + 4 * half + (v & 3);
        const int64_t m = m0 + row;
        const int64_t np = n0 + wn * UN * 16 + j * 16 + (j32 >> 1);
        if (m < M && np < N) out[(m * N + np) * 2 + bc] = acc[i][j][v];
      }
}

__global__ __launch_bounds__(kThreads) void k_reduce(ReduceArgs a) {
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

// ---------------------------------------------------------------------------------
// slices
__global__ __launch_bounds__(kThreads) void k_slice_leaves(SliceLeafArgs a, int64_t per_slice) {
  const int64_t base = *a.base;
  const int64_t total = per_slice * a.nb;
  for (int64_t g = int64_t(blockIdx.x) * kThreads + threadIdx.x; g < total;
       g += int64_t(gridDim.x) * kThreads) {
    const int64_t sl = g / per_slice, gg = g - sl * per_slice;
    const uint64_t sigma = a.slice_ids[base + sl];
    int e = 0;
    while (e + 1 < a.n_entries && a.prefix[e + 1] <= gg) ++e;
    const SliceLeafEntry& t = a.table[e];
    const int64_t o = gg - a.prefix[e];
    const int64_t row = o >> t.dense_out;
    int64_t d = o & ((int64_t(1) << t.dense_out) - 1);
    for (int j = 0; j < t.n_sl; ++j) {
      const int p = t.pos[j];
      const int64_t v = (sigma >> t.bit[j]) & 1;
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
      o.x += double(v.x);
      o.y += double(v.y);
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

int grid_for(int64_t work, int64_t per_block, int64_t cap = 8192) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return int(g);
}

template <int NK, int NN>
hipError_t launch_stream_t(const StreamArgs& a, hipStream_t s) {
  const int64_t total = (a.rows << a.n_m) * a.nb;
  hipLaunchKernelGGL((k_stream<NK, NN>), dim3(grid_for(total, kThreads, 65536)), dim3(kThreads), 0,
                     s, a);
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
  if (!a.a_mfast && !a.b_nfast)
    hipLaunchKernelGGL((k_gemm<WM, WN, UM, UN, BK, false, false>), grid, dim3(kThreads), 0, s, a);
  else if (a.a_mfast && !a.b_nfast)
    hipLaunchKernelGGL((k_gemm<WM, WN, UM, UN, BK, true, false>), grid, dim3(kThreads), 0, s, a);
  else if (!a.a_mfast && a.b_nfast)
    hipLaunchKernelGGL((k_gemm<WM, WN, UM, UN, BK, false, true>), grid, dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL((k_gemm<WM, WN, UM, UN, BK, true, true>), grid, dim3(kThreads), 0, s, a);
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
// 1 = 128 x 16 (4x1 waves, one MFMA tile each), 2 = 64 x 32 (2x2 waves, one tile each).
hipError_t launch_gemm(const GemmArgs& a, hipStream_t s) {
  switch (a.config) {
    case 0: return launch_gemm_cfg<2, 2, 2, 2, 16>(a, s);
    case 1: return launch_gemm_cfg<4, 1, 1, 1, 16>(a, s);
    case 2: return launch_gemm_cfg<2, 2, 1, 1, 16>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s) {
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
