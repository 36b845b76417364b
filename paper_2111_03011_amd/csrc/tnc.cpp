// libtnc host runtime: C ABI, validation, step compiler, workspace planner, executor.
//
// The contraction of one slice is compiled once into a list of kernel launches:
//   * leaves carrying sliced bonds are instantiated per slice (paper, Appendix B.2);
//   * every path pair (Appendix E format) becomes either a fused small-operand stream or a
//     complex GEMM that reads both operands in their stored layouts (no permute is ever
//     issued), optionally split along K with a fixed-order reduction;
//   * tensors that carry closed final qubits keep one row per distinct restriction of the
//     requested bitstrings (Appendix A: only the configurations some target needs), and
//     a contraction of two such tensors gathers the matching operand rows;
//   * the last tensor is added in FP64 to psi_hat (the sum over slices, Results).
// Steps whose subtree holds no sliced leaf are identical in every slice and run once per
// call.  All device memory is the caller's workspace: a constants block (leaves, row maps,
// tables) followed by an arena whose buffers are packed by lifetime.
#include "tnc.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <deque>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <stdexcept>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "tnc_internal.h"
#include "tnc_kernels.h"

using namespace tnc;

namespace {

thread_local std::string g_err;

struct Error {
  tnc_status code;
  std::string msg;
};

[[noreturn]] void fail(tnc_status c, const std::string& m) { throw Error{c, m}; }

#define HIPCHK(x)                                                                   \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) fail(TNC_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class F>
tnc_status guard(F&& f) {
  try {
    f();
    g_err.clear();
    return TNC_OK;
  } catch (const Error& e) {
    g_err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host out of memory";
    return TNC_E_OOM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return TNC_E_INTERNAL;
  }
}

constexpr uint64_t kAlign = 256;
uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

}  // namespace

// ------------------------------------------------------------------------------------
struct tnc_net_s {
  int device = 0;
  int n_qubits = 0;
  std::vector<std::vector<int32_t>> labels;
  std::vector<std::vector<double>> data;
  std::vector<int32_t> out_label;
  std::map<int32_t, std::vector<int>> holders;
  bool has_path = false;
  std::vector<std::pair<int, int>> path;
  bool has_slices = false;
  std::vector<int32_t> sliced;
  std::vector<uint64_t> slice_ids;   // two 64-bit words per id (bits 0-63, 64-127)
  bool has_targets = false;
  std::vector<int32_t> open;
  std::vector<uint64_t> closed;
};

namespace {

enum Kind { K_PERMUTE = 0, K_GEMM = 1, K_STREAM = 2, K_LEAVES = 3, K_SUM = 4, K_REDUCE = 5, K_SPLIT = 6 };
constexpr int kKinds = 7;
// kind K_SPLIT: the clearing of a block of scale records before their producers fold
// their outputs' largest components into them
enum SplitOp { SPLIT_ZERO = 2 };

// Scale records (see kRecWords) live in three blocks: constants (the leaves' largest
// components, measured on the host, exponent 0), one copy for the slice-invariant tensors
// (cleared at the start of every call) and one per slice copy of a batch for the
// slice-dependent ones (cleared at the start of every batch).
enum RecBlock { REC_CONST = 0, REC_INV = 1, REC_DEP = 2 };
struct Rec {
  int block = REC_CONST;
  int64_t index = 0;          // record number inside its block
  bool per_slice = false;     // one record per slice copy (else one shared by every slice)
};

struct Buf {
  uint64_t bytes = 0;         // all copies
  uint64_t elems = 0;         // complex64 elements of one copy
  bool per_slice = false;     // one copy per slice of a batch
  bool is_const = false;
  uint64_t off = 0;       // absolute byte offset in the workspace
  int t0 = INT_MAX, t1 = -1;
  bool to_end = false;    // produced once, read by every slice
};

struct Launch {
  int kind = 0;
  bool inv = false;
  std::vector<int> bufs;  // buffers touched (for lifetimes)
  int b_in0 = -1, b_in1 = -1, b_out = -1, b_tmp = -1;
  int64_t g0 = -1, g1 = -1;   // byte offsets of row gathers in the constants block
  int64_t stk_off = -1, perm_off = -1;   // row-stacking tables (GEMM), same block
  int rec_in0 = -1, rec_in1 = -1, rec_out = -1;   // scale records of the operands and result
  bool shared = false;        // slice-dependent, but the same for every slice of a batch
  int split_op = 0;                      // K_SPLIT: SPLIT_ZERO
  int64_t n_elems = 0;        // words per slice copy (record clearing)
  bool enabled = true;        // a split-K reduction is switched off when tuning drops split-K
  int max_splits = 1;         // split-K factor the partial buffer was sized for
  StreamArgs st{};
  GemmArgs gm{};
  ReduceArgs rd{};
  tnc_step_info info{};
};

struct TState {
  std::vector<int32_t> dense;   // slowest first
  uint64_t q = 0;
  std::vector<uint64_t> keys;
  bool dep = false;
  int buf = -1;
  int rec = -1;                 // scale record
  uint64_t dbits[2] = {0, 0};   // slice-id bits (sliced labels) the tensor depends on
  bool shared = false;          // dep, and none of its bits varies inside a batch
  bool per_slice() const { return dep && !shared; }
  bool alive = true;
  int64_t rows() const { return int64_t(keys.size()); }
  int64_t elems() const { return rows() << dense.size(); }
};

struct TimingRec {
  int kind;
  int index;   // launch index (invariant launches first), -1 if not one of the plan's
  double bytes, flops;
  hipEvent_t e0, e1;
};

}  // namespace

struct tnc_plan_s {
  int device = 0;
  int n_qubits = 0;
  tnc_precision precision = TNC_C64;
  int64_t L = 1;
  int n_open = 0;
  std::vector<int32_t> open;
  std::vector<uint64_t> closed;
  std::vector<uint64_t> slice_ids;   // two words per id
  int64_t n_slices() const { return int64_t(slice_ids.size() / 2); }

  std::vector<Buf> bufs;
  std::vector<Rec> recs;
  int rec_buf[3] = {-1, -1, -1};     // buffers of the three record blocks
  int64_t rec_count[3] = {0, 0, 0};  // records per block (per slice copy)
  std::vector<uint8_t> consts;
  uint64_t consts_bytes = 0, ws_bytes = 0;
  std::vector<Launch> inv, dep;

  // slice leaves
  std::vector<SliceLeafEntry> sl_table;
  std::vector<int64_t> sl_prefix;
  int64_t sl_total = 0;
  int64_t sl_table_off = -1, sl_prefix_off = -1;
  int64_t slice_ids_off = 0;
  // final sum
  SliceSumArgs ss{};
  int final_buf = -1;
  int64_t row_of_off = 0;
  // sampling and norm scratch
  int64_t closed_off = 0, open_off = 0;
  int norm_parts = 1024;
  int b_norm = -1, b_cum = -1, b_samples = -1, b_counter = -1, b_totals = -1;
  int batch = 1;
  // slice-id bits that vary inside some batch of the slice list (batches of `batch`
  // consecutive ids, or shorter runs, see Exec::run_length); a dependent step whose bits
  // avoid them is computed once per batch
  uint64_t vary[2] = {~uint64_t(0), ~uint64_t(0)};
  double flops_shared = 0;   // algorithmic flops of the once-per-batch steps (one copy)
  // captured program of one full batch (per workspace and amplitude buffer)
  hipGraphExec_t graph = nullptr;
  hipStream_t capture_stream = nullptr;
  const void* graph_ws = nullptr;
  const void* graph_amps = nullptr;
  int64_t sample_chunk = 0;

  double flops_slice = 0, bytes_slice = 0, flops_inv = 0, bytes_inv = 0;
  int n_steps = 0;

  const void* uploaded_ws = nullptr;

  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<TimingRec> pending;
  double t_ms[kKinds] = {}, t_bytes[kKinds] = {}, t_flops[kKinds] = {};
  std::vector<double> l_ms;      // per launch index, summed over timed launches
  std::vector<int64_t> l_n;
  int64_t t_n[kKinds] = {};
  ~tnc_plan_s() {
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    if (graph) (void)hipGraphExecDestroy(graph);
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
  }
};

// ------------------------------------------------------------------------------------
// helpers
namespace {

std::vector<uint64_t> row_keys(const std::vector<uint64_t>& closed, uint64_t q) {
  std::vector<uint64_t> k;
  if (q == 0) return {0};
  k.reserve(closed.size());
  for (uint64_t c : closed) k.push_back(c & q);
  std::sort(k.begin(), k.end());
  k.erase(std::unique(k.begin(), k.end()), k.end());
  return k;
}

int pos_of(const std::vector<int32_t>& dense, int32_t label) {
  for (size_t i = 0; i < dense.size(); ++i)
    if (dense[i] == label) return int(dense.size() - 1 - i);
  return -1;
}

struct Compiler {
  tnc_net_s& net;
  tnc_plan_s& plan;
  std::vector<TState> T;
  std::set<int32_t> sliced_set;
  std::map<int32_t, int> sliced_bit;

  Compiler(tnc_net_s& n, tnc_plan_s& p) : net(n), plan(p) {}

  int new_buf(uint64_t bytes, bool is_const = false, bool per_slice = false) {
    Buf b;
    b.elems = bytes / 8;
    b.per_slice = per_slice;
    const uint64_t copies = per_slice ? uint64_t(plan.batch) : 1;
    b.bytes = align_up(std::max<uint64_t>(bytes * copies, 8));
    b.is_const = is_const;
    plan.bufs.push_back(b);
    return int(plan.bufs.size() - 1);
  }

  int64_t sstride(int b) const {
    return plan.bufs[b].per_slice ? int64_t(plan.bufs[b].elems) : 0;
  }

  int64_t add_const(const void* p, uint64_t bytes) {
    const uint64_t off = align_up(plan.consts.size());
    plan.consts.resize(off + bytes);
    if (bytes) std::memcpy(plan.consts.data() + off, p, bytes);
    plan.consts.resize(align_up(plan.consts.size()));
    return int64_t(off);
  }

  int const_buf(const void* p, uint64_t bytes) {
    const int64_t off = add_const(p, bytes);
    const int b = new_buf(bytes, true);
    plan.bufs[b].off = uint64_t(off);
    return b;
  }

  std::vector<Launch>& list(bool inv) { return inv ? plan.inv : plan.dep; }

  // gather map of an operand into output rows; -1 = none needed
  int64_t gather(const TState& op, const TState& out) {
    if (op.q == out.q || op.q == 0) return -1;
    std::vector<int32_t> g(out.keys.size());
    for (size_t r = 0; r < out.keys.size(); ++r) {
      const uint64_t k = out.keys[r] & op.q;
      auto it = std::lower_bound(op.keys.begin(), op.keys.end(), k);
      if (it == op.keys.end() || *it != k) fail(TNC_E_INTERNAL, "row map lookup failed");
      g[r] = int32_t(it - op.keys.begin());
    }
    return add_const(g.data(), g.size() * sizeof(int32_t));
  }

  void leaves() {
    const int n = net.n_qubits;
    std::set<int32_t> open_set(net.open.begin(), net.open.end());
    std::map<int32_t, int> closed_leg;
    for (int q = 0; q < n; ++q)
      if (!open_set.count(q)) closed_leg[net.out_label[q]] = q;
    for (size_t b = 0; b < net.sliced.size(); ++b) {
      sliced_set.insert(net.sliced[b]);
      sliced_bit[net.sliced[b]] = int(b);
    }
    T.resize(net.labels.size());
    for (size_t t = 0; t < net.labels.size(); ++t) {
      const auto& lab = net.labels[t];
      const int rank = int(lab.size());
      TState s;
      std::vector<int32_t> full;       // dense incl. sliced
      std::vector<int> full_w, cl_w, cl_q;
      for (int p = 0; p < rank; ++p) {
        const int64_t w = int64_t(1) << (rank - 1 - p);
        auto it = closed_leg.find(lab[p]);
        if (it != closed_leg.end()) {
          s.q |= uint64_t(1) << (n - 1 - it->second);
          cl_w.push_back(int(rank - 1 - p));
          cl_q.push_back(it->second);
        } else {
          full.push_back(lab[p]);
          full_w.push_back(int(rank - 1 - p));
        }
        (void)w;
      }
      s.keys = row_keys(net.closed, s.q);
      const int df = int(full.size());
      std::vector<float> host(size_t(s.rows()) * (size_t(1) << df) * 2);
      for (int64_t r = 0; r < s.rows(); ++r) {
        int64_t base = 0;
        for (size_t c = 0; c < cl_q.size(); ++c)
          if ((s.keys[r] >> (n - 1 - cl_q[c])) & 1) base += int64_t(1) << cl_w[c];
        for (int64_t d = 0; d < (int64_t(1) << df); ++d) {
          int64_t o = base;
          for (int j = 0; j < df; ++j)
            if ((d >> (df - 1 - j)) & 1) o += int64_t(1) << full_w[j];
          const size_t h = size_t((r << df) + d) * 2;
          host[h] = float(net.data[t][2 * o]);
          host[h + 1] = float(net.data[t][2 * o + 1]);
        }
      }
      std::vector<int32_t> dense;
      std::vector<std::pair<int, int>> sl;   // (position in full dense, slice bit)
      for (int j = 0; j < df; ++j) {
        if (sliced_set.count(full[j]))
          sl.push_back({df - 1 - j, sliced_bit[full[j]]});
        else
          dense.push_back(full[j]);
      }
      s.dense = dense;
      float mx = 0.f;
      for (float v : host) mx = std::max(mx, std::fabs(v));
      uint32_t bits;
      std::memcpy(&bits, &mx, 4);
      s.rec = new_rec(REC_CONST, false);
      const_amax.push_back(bits);
      if (sl.empty()) {
        s.buf = const_buf(host.data(), host.size() * sizeof(float));
      } else {
        if (sl.size() > 8) fail(TNC_E_UNSUPPORTED, "a leaf holds more than 8 sliced labels");
        std::sort(sl.begin(), sl.end());
        SliceLeafEntry e{};
        e.src_off = add_const(host.data(), host.size() * sizeof(float)) / 8;
        e.elems_out = s.rows() << dense.size();
        e.dense_out = int32_t(dense.size());
        e.n_sl = int32_t(sl.size());
        for (size_t j = 0; j < sl.size(); ++j) {
          e.pos[j] = int8_t(sl[j].first);
          e.bit[j] = int8_t(sl[j].second);
        }
        s.dep = true;
        for (size_t j = 0; j < sl.size(); ++j) s.dbits[sl[j].second >> 6] |= uint64_t(1) << (sl[j].second & 63);
        s.buf = new_buf(uint64_t(e.elems_out) * 8, false, true);
        e.dst_off = s.buf;    // resolved after packing
        plan.sl_table.push_back(e);
      }
      T[t] = std::move(s);
    }
    if (!plan.sl_table.empty()) {
      Launch L;
      L.kind = K_LEAVES;
      L.inv = false;
      for (auto& e : plan.sl_table) L.bufs.push_back(int(e.dst_off));
      int64_t tot = 0;
      plan.sl_prefix.push_back(0);
      for (auto& e : plan.sl_table) {
        tot += e.elems_out;
        plan.sl_prefix.push_back(tot);
      }
      plan.sl_total = tot;
      L.info.kind = K_LEAVES;
      L.info.bytes = 16.0 * double(tot);
      plan.dep.push_back(L);
    }
  }

  void account(const Launch& L) {
    if (L.inv) {
      plan.flops_inv += L.info.flops;
      plan.bytes_inv += L.info.bytes;
    } else {
      plan.flops_slice += L.info.flops;
      plan.bytes_slice += L.info.bytes;
      if (L.shared) plan.flops_shared += L.info.flops;
    }
  }

  // Tile configuration and split-K.  Debug overrides: TNC_GEMM_CONFIG forces a tile
  // configuration, TNC_SPLITK_BLOCKS sets the workgroup count split-K aims for.
  // Row stacking of output rows that share one Q row: perm sorts the output rows by their
  // Q row, and within one Q row by their P row; each 128-row block holds up to 128 / M rows
  // of one Q row (start, count, Q row).  The blocks are then ordered by the P row of their
  // first output row, so that blocks of different Q rows that read the same P rows are
  // numbered, hence placed on one XCD and run, close together (a P row used by several
  // output rows is then read from HBM about once and served from that XCD's L2).
  // Returns the fraction of the stacked M extent that holds real rows.
  static double stack_rows(const TState& P, const TState& Q, const TState& C, int64_t M,
                           std::vector<int32_t>& stk, std::vector<int32_t>& perm) {
    const int64_t rows = C.rows();
    auto row_of = [&](const TState& S, std::vector<int32_t>& out) {
      out.assign(size_t(rows), 0);
      if (S.q == 0) return;
      for (int64_t r = 0; r < rows; ++r) {
        const uint64_t k = C.keys[size_t(r)] & S.q;
        out[size_t(r)] = int32_t(std::lower_bound(S.keys.begin(), S.keys.end(), k) - S.keys.begin());
      }
    };
    std::vector<int32_t> qrow, prow;
    row_of(Q, qrow);
    row_of(P, prow);
    perm.resize(size_t(rows));
    for (int64_t r = 0; r < rows; ++r) perm[size_t(r)] = int32_t(r);
    std::stable_sort(perm.begin(), perm.end(), [&](int32_t x, int32_t y) {
      return qrow[size_t(x)] != qrow[size_t(y)] ? qrow[size_t(x)] < qrow[size_t(y)]
                                                : prow[size_t(x)] < prow[size_t(y)];
    });
    std::vector<std::array<int32_t, 3>> blocks;
    const int64_t per = 128 / M;
    for (int64_t i = 0; i < rows;) {
      int64_t j = i;
      const int32_t q0 = qrow[size_t(perm[size_t(i)])];
      while (j < rows && j - i < per && qrow[size_t(perm[size_t(j)])] == q0) ++j;
      blocks.push_back({int32_t(i), int32_t(j - i), q0});
      i = j;
    }
    std::stable_sort(blocks.begin(), blocks.end(),
                     [&](const std::array<int32_t, 3>& x, const std::array<int32_t, 3>& y) {
                       return prow[size_t(perm[size_t(x[0])])] < prow[size_t(perm[size_t(y[0])])];
                     });
    stk.clear();
    for (const auto& b : blocks) stk.insert(stk.end(), {b[0], b[1], b[2]});
    return double(rows * M) / (double(stk.size() / 3) * 128.0);
  }

  // Estimated fraction of the MFMA tile work that is useful, for P on the M side
  static double tile_fill(const TState& P, const TState& Q, const TState& C, int nm, int nn) {
    const int64_t M = int64_t(1) << nm, N = int64_t(1) << nn, rows = C.rows();
    static const int64_t kBM[kConfigs] = {128, 128, 64, 128, 128, 128, 256, 128, 256};
    static const int64_t kBN[kConfigs] = {64, 16, 32, 128, 32, 8, 512, 128, 64};
    int64_t m_eff = M;
    if (rows > 1 && Q.rows() == 1 && P.q == C.q && M >= 128) m_eff = M * rows;
    double fm;
    const int cfg = (N <= 16) ? 1 : (m_eff <= 64 ? 2 : (N <= 32 ? 4 : 0));
    fm = std::min(1.0, double(m_eff) / double(kBM[cfg]));
    if (m_eff < 128 && rows > 1 && Q.rows() < rows && stacking_enabled()) {
      std::vector<int32_t> stk, perm;
      fm = std::max(fm, stack_rows(P, Q, C, M, stk, perm));
    }
    // an N <= 8 step is charged as a 16-wide tile: its 16x16x4 tiles reuse operands less
    // than a stacked orientation of the same step would
    const int cfg_n = (N <= 16) ? 1 : (N <= 32 ? 4 : 0);
    return fm * std::min(1.0, double(N) / double(kBN[cfg_n]));
  }

  // GEMM tile configurations (see launch_gemm); 6 is the short-K vector kernel, 7 and 8
  // the eight-wave 128 x 128 and 256 x 64 tiles of the split-precision forms
  static constexpr int kConfigs = 9;

  // read at every plan compile, so that one process can build plans both ways
  static bool stacking_enabled() { return std::getenv("TNC_NO_STACK") == nullptr; }

  // the short-K kernel (configuration 6) takes K <= 16 without row stacking; the eight-wave
  // tiles (configurations 7, 8) any precision without row stacking
  static bool outer_ok(const GemmArgs& g, bool stacked) { return g.nk <= 4 && !stacked; }
  static bool big_ok(const GemmArgs& g, bool stacked) { (void)g; return !stacked; }

  static void choose_tiles(GemmArgs& g, int64_t M, int64_t N, int64_t Kd, int64_t rows,
                           bool stacked) {
    static const int group = std::getenv("TNC_GEMM_GROUP") ? std::atoi(std::getenv("TNC_GEMM_GROUP")) : 4;
    g.group_m = group;
    const char* force = std::getenv("TNC_GEMM_CONFIG");
    const char* blocks_env = std::getenv("TNC_SPLITK_BLOCKS");
    const int64_t target = blocks_env ? std::atoll(blocks_env) : 2048;
    g.config = (N <= 8) ? 5 : (N <= 16) ? 1 : (M <= 64 ? 2 : (N <= 32 ? 4 : 0));
    // short contraction, wide output of at least 2^22 elements: bound by writing C
    if (outer_ok(g, stacked) && N >= 64 && double(M) * double(N) * double(rows) >= 4194304.0)
      g.config = 6;
    if (force) {
      const int f = std::min(kConfigs - 1, std::max(0, std::atoi(force)));
      if ((f != 6 || outer_ok(g, stacked)) && (f < 7 || big_ok(g, stacked))) g.config = f;
    }
    static const int64_t kBM[kConfigs] = {128, 128, 64, 128, 128, 128, 256, 128, 256};
    static const int64_t kBN[kConfigs] = {64, 16, 32, 128, 32, 8, 512, 128, 64};
    const int64_t BM = kBM[g.config], BN = kBN[g.config];
    const int64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN) * rows;
    g.k_splits = 1;
    g.k_chunk = Kd;
    if (tiles * 4 <= target && Kd >= 512) {
      int64_t s = 1;
      while (tiles * s * 2 <= target && Kd / (s * 2) >= 256) s *= 2;
      g.k_splits = int(s);
      g.k_chunk = Kd / s;
    }
  }

  // a new scale record: slice-invariant tensors in the per-call block, slice-dependent
  // ones in the per-batch block (one per slice copy unless shared by the batch)
  int new_rec(int block, bool per_slice) {
    Rec r;
    r.block = block;
    r.index = plan.rec_count[block]++;
    r.per_slice = per_slice;
    plan.recs.push_back(r);
    return int(plan.recs.size() - 1);
  }
  std::vector<uint32_t> const_amax;   // largest component of each constant record

  // the record blocks and their clearing launches, once every tensor has its record
  void finish_records() {
    std::vector<uint32_t> words(size_t(plan.rec_count[REC_CONST]) * kRecWords, 0u);
    for (size_t i = 0; i < const_amax.size(); ++i)
      for (int j = 0; j < kAmaxSlots; ++j) words[i * kRecWords + j] = const_amax[i];
    if (!words.empty()) plan.rec_buf[REC_CONST] = const_buf(words.data(), words.size() * 4);
    for (int blk : {REC_INV, REC_DEP}) {
      if (plan.rec_count[blk] == 0) continue;
      const uint64_t words_per_copy = uint64_t(plan.rec_count[blk]) * kRecWords;
      // not listed in any launch's buffers: kept for the whole call
      plan.rec_buf[blk] = new_buf(words_per_copy * 4, false, blk == REC_DEP);
      Launch Z;
      Z.kind = K_SPLIT;
      Z.split_op = SPLIT_ZERO;
      Z.inv = blk == REC_INV;
      Z.b_out = plan.rec_buf[blk];
      Z.n_elems = int64_t(words_per_copy);
      Z.info = tnc_step_info{K_SPLIT, Z.inv, 1, int64_t(words_per_copy), 0, 0, 0.0,
                             4.0 * double(words_per_copy)};
      std::vector<Launch>& lst = list(Z.inv);
      lst.insert(lst.begin(), Z);
    }
  }

  TState step(TState& A, TState& B) {
    TState C;
    C.dep = A.dep || B.dep;
    const bool inv = !C.dep;
    C.dbits[0] = A.dbits[0] | B.dbits[0];
    C.dbits[1] = A.dbits[1] | B.dbits[1];
    C.shared = C.dep && !(C.dbits[0] & plan.vary[0]) && !(C.dbits[1] & plan.vary[1]);
    const bool ps = C.per_slice();
    C.q = A.q | B.q;
    C.keys = row_keys(net.closed, C.q);
    std::set<int32_t> sa(A.dense.begin(), A.dense.end()), sb(B.dense.begin(), B.dense.end());
    std::vector<int32_t> K, MA, NB;
    for (auto x : A.dense) (sb.count(x) ? K : MA).push_back(x);
    for (auto x : B.dense)
      if (!sa.count(x)) NB.push_back(x);
    const int nk = int(K.size());
    const double macs = double(C.rows()) * std::ldexp(1.0, int(MA.size() + NB.size() + K.size()));

    // fused stream: one operand small enough to sit in registers/LDS.  K up to 16 by
    // default: from K = 32 on, the matrix-core GEMM is faster on the 53-qubit share's
    // row steps (K = 64 ran at about 27 TFLOP/s as a stream); TNC_STREAM_MAX_NK (up to 6,
    // read at every compile) moves the limit
    const char* snk = std::getenv("TNC_STREAM_MAX_NK");
    const int stream_max_nk = snk ? std::min(6, std::atoi(snk)) : 4;
    auto stream_ok = [&](const TState& S, const std::vector<int32_t>& Sfree) {
      return nk <= stream_max_nk && int(Sfree.size()) <= 4;
    };
    const bool a_small = stream_ok(A, MA), b_small = stream_ok(B, NB);
    if (a_small || b_small) {
      bool x_is_a;
      if (a_small && b_small) x_is_a = A.elems() >= B.elems();
      else x_is_a = b_small;
      TState& X = x_is_a ? A : B;
      TState& S = x_is_a ? B : A;
      const std::vector<int32_t>& MX = x_is_a ? MA : NB;
      const std::vector<int32_t>& NS = x_is_a ? NB : MA;
      Launch L;
      L.kind = K_STREAM;
      L.inv = inv;
      L.shared = C.shared;
      StreamArgs& a = L.st;
      a.rows = C.rows();
      a.x_rows = X.rows();
      a.s_rows = S.rows();
      a.x_row_stride = int64_t(1) << X.dense.size();
      a.s_row_stride = int64_t(1) << S.dense.size();
      a.n_m = int(MX.size());
      a.nk = nk;
      a.nn = int(NS.size());
      a.c_row_stride = int64_t(1) << (a.n_m + a.nn);
      std::vector<int> kins;
      for (int j = 0; j < nk; ++j) {
        a.x_kpos[j] = int8_t(pos_of(X.dense, K[j]));
        a.s_kpos[j] = int8_t(pos_of(S.dense, K[j]));
        kins.push_back(a.x_kpos[j]);
      }
      std::sort(kins.begin(), kins.end());
      for (int j = 0; j < nk; ++j) a.x_kins[j] = int8_t(kins[j]);
      for (int j = 0; j < a.nn; ++j) a.s_npos[j] = int8_t(pos_of(S.dense, NS[NS.size() - 1 - j]));
      C.dense = MX;
      C.dense.insert(C.dense.end(), NS.begin(), NS.end());
      C.buf = new_buf(uint64_t(C.elems()) * 8, false, ps);
      C.rec = new_rec(inv ? REC_INV : REC_DEP, ps);
      L.rec_in0 = X.rec;
      L.rec_in1 = S.rec;
      L.rec_out = C.rec;
      a.x_slice_stride = sstride(X.buf);
      a.s_slice_stride = sstride(S.buf);
      a.c_slice_stride = sstride(C.buf);
      L.b_in0 = X.buf;
      L.b_in1 = S.buf;
      L.b_out = C.buf;
      L.g0 = gather(X, C);
      L.g1 = gather(S, C);
      L.bufs = {X.buf, S.buf, C.buf};
      L.info = tnc_step_info{K_STREAM, inv, C.rows(), int64_t(1) << a.n_m, int64_t(1) << a.nn,
                             int64_t(1) << nk, 8.0 * macs,
                             8.0 * double(X.elems() + S.elems() + C.elems())};
      account(L);
      list(inv).push_back(L);
      return C;
    }

    // GEMM: P supplies the M side, Q the N side.  The kernels address one operand row
    // with 32-bit offsets.
    if (A.dense.size() > 31 || B.dense.size() > 31)
      fail(TNC_E_UNSUPPORTED, "a GEMM operand row holds more than 2^31 elements");
    if (nk > 28) fail(TNC_E_UNSUPPORTED, "a GEMM contracts more than 28 labels (K > 2^28)");
    // P supplies the M side: by default the operand with more rows x free elements; the
    // other orientation is taken when its tiles are clearly fuller (row stacking needs the
    // operand whose rows are shared on the N side)
    bool p_is_a = (double(A.rows()) * std::ldexp(1.0, int(MA.size()))) >=
                  (double(B.rows()) * std::ldexp(1.0, int(NB.size())));
    if (C.rows() > 1) {
      const double f_keep = p_is_a ? tile_fill(A, B, C, int(MA.size()), int(NB.size()))
                                   : tile_fill(B, A, C, int(NB.size()), int(MA.size()));
      const double f_swap = p_is_a ? tile_fill(B, A, C, int(NB.size()), int(MA.size()))
                                   : tile_fill(A, B, C, int(MA.size()), int(NB.size()));
      if (f_swap > 1.2 * f_keep) p_is_a = !p_is_a;
    }
    TState& P = p_is_a ? A : B;
    TState& Q = p_is_a ? B : A;
    const std::vector<int32_t>& MP = p_is_a ? MA : NB;
    const std::vector<int32_t>& NQ = p_is_a ? NB : MA;
    std::vector<int32_t> KP, KQ;   // K in P's / Q's order
    for (auto x : P.dense)
      if (std::find(K.begin(), K.end(), x) != K.end()) KP.push_back(x);
    for (auto x : Q.dense)
      if (std::find(K.begin(), K.end(), x) != K.end()) KQ.push_back(x);
    auto cat = [](const std::vector<int32_t>& x, const std::vector<int32_t>& y) {
      std::vector<int32_t> r = x;
      r.insert(r.end(), y.begin(), y.end());
      return r;
    };
    // the logical k order follows the larger operand, so its loads stay contiguous
    const std::vector<int32_t>& Kord = (P.elems() >= Q.elems()) ? KP : KQ;
    Launch L;
    L.kind = K_GEMM;
    L.inv = inv;
    L.shared = C.shared;
    GemmArgs& g = L.gm;
    const int nm = int(MP.size()), nn = int(NQ.size());
    int64_t M = int64_t(1) << nm, N = int64_t(1) << nn, Kd = int64_t(1) << nk;
    int64_t rows = C.rows();
    g.nm = nm;
    g.nk = nk;
    g.nn = nn;
    for (int j = 0; j < nm; ++j) g.a_mpos[j] = int8_t(pos_of(P.dense, MP[nm - 1 - j]));
    for (int j = 0; j < nk; ++j) {
      g.a_kpos[j] = int8_t(pos_of(P.dense, Kord[nk - 1 - j]));
      g.b_kpos[j] = int8_t(pos_of(Q.dense, Kord[nk - 1 - j]));
    }
    for (int j = 0; j < nn; ++j) g.b_npos[j] = int8_t(pos_of(Q.dense, NQ[nn - 1 - j]));
    g.a_mfast = (!P.dense.empty() && std::find(MP.begin(), MP.end(), P.dense.back()) != MP.end());
    g.b_nfast = (!Q.dense.empty() && std::find(NQ.begin(), NQ.end(), Q.dense.back()) != NQ.end());
    int pbuf = P.buf, qbuf = Q.buf;
    L.g0 = gather(P, C);
    L.g1 = gather(Q, C);
    g.a_rows = P.rows();
    g.b_rows = Q.rows();
    g.a_row_stride = int64_t(1) << P.dense.size();
    g.b_row_stride = int64_t(1) << Q.dense.size();
    // rows folded into M when Q is shared by every row and P's rows line up with C's
    // (a tile never straddles two rows: the per-row M is at least the largest tile)
    const int64_t rows_c = rows, m_c = M;
    int64_t c_row_stride = M * N;
    if (rows > 1 && Q.rows() == 1 && P.q == C.q && M >= 128) {
      g.fold = 1;
      g.fold_stride = g.a_row_stride;
      M *= rows;
      rows = 1;
      g.a_rows = 1;
      g.a_row_stride = 0;
      c_row_stride = M * N;
    }
    // row stacking: output rows whose M is below a tile and that share one Q row are
    // stacked along M, 128 >> nm rows per 128-row block
    std::vector<int32_t> stk, perm;
    if (!g.fold && rows > 1 && M < 128 && Q.rows() < rows && stacking_enabled() &&
        double(P.elems()) < 2147483648.0) {
      // tile fill in both directions: unstacked, the better of the 64 x 32 tile and the
      // 128-row tiles (128 x 8 / 16 / 32 / 64 by N); stacked, the 128-row tile
      const double nd = double(N);
      const double n128 = std::min(1.0, nd / (N <= 8 ? 8.0 : N <= 16 ? 16.0 : N <= 32 ? 32.0 : 64.0));
      const double fill_plain = std::max(std::min(1.0, double(M) / 64.0) * std::min(1.0, nd / 32.0),
                                         std::min(1.0, double(M) / 128.0) * n128);
      const double fill_stacked = stack_rows(P, Q, C, M, stk, perm) * n128;
      if (fill_stacked > 1.25 * fill_plain) {
        M = int64_t(stk.size() / 3) * 128;
        rows = 1;
      } else {
        stk.clear();
        perm.clear();
      }
    }
    g.M = M;
    g.N = N;
    g.K = Kd;
    g.rows = rows;
    g.c_row_stride = c_row_stride;
    g.precision = 0;
    if (plan.precision == TNC_FP16X3) g.precision = 3;
    if (plan.precision == TNC_BF16X3) g.precision = 1;
    choose_tiles(g, M, N, Kd, rows, !stk.empty());
    if (!stk.empty()) {
      g.k_splits = 1;   // the split-K reduce assumes C in the launch's own layout
      g.k_chunk = Kd;
      L.stk_off = add_const(stk.data(), stk.size() * sizeof(int32_t));
      L.perm_off = add_const(perm.data(), perm.size() * sizeof(int32_t));
    }
    // no 8-wide split tile; rows of narrow long-K products keep the FP32 narrow-row kernel
    if (plan.precision != TNC_C64 && g.config == 5 && !gemm_rows_narrow_fits(g, !stk.empty()))
      g.config = 1;
    C.rec = new_rec(inv ? REC_INV : REC_DEP, ps);
    L.rec_in0 = P.rec;
    L.rec_in1 = Q.rec;
    L.rec_out = C.rec;
    C.dense = cat(MP, NQ);
    C.buf = new_buf(uint64_t(C.elems()) * 8, false, ps);
    g.a_slice_stride = sstride(pbuf);
    g.b_slice_stride = sstride(qbuf);
    g.c_slice_stride = sstride(C.buf);
    L.b_in0 = pbuf;
    L.b_in1 = qbuf;
    L.b_out = C.buf;
    L.bufs = {pbuf, qbuf, C.buf};
    int part = -1;
    L.max_splits = g.k_splits;
    if (g.k_splits > 1) {
      part = new_buf(uint64_t(g.k_splits) * uint64_t(rows) * uint64_t(M) * uint64_t(N) * 8, false,
                     ps);
      L.b_tmp = part;
      L.bufs.push_back(part);
    }
    L.info = tnc_step_info{K_GEMM, inv, rows_c, m_c, N, Kd, 8.0 * macs,
                           8.0 * double(P.elems() + Q.elems() + C.elems())};
    account(L);
    list(inv).push_back(L);
    if (part >= 0) {
      Launch R;
      R.kind = K_REDUCE;
      R.inv = inv;
      R.shared = C.shared;
      R.rd.elems = rows * M * N;
      R.rd.splits = g.k_splits;
      R.b_in0 = part;
      R.b_out = C.buf;
      R.bufs = {part, C.buf};
      R.rd.slice_elems = rows * M * N;
      R.rec_out = C.rec;
      R.info = tnc_step_info{K_REDUCE, inv, rows, M, N, 0, 0.0,
                             8.0 * double(g.k_splits + 1) * double(rows * M * N)};
      account(R);
      list(inv).push_back(R);
    }
    return C;
  }

  void run() {
    leaves();
    for (auto& pr : net.path) {
      TState& A = T[pr.first];
      TState& B = T[pr.second];
      TState C = step(A, B);
      B.alive = false;
      A = std::move(C);
      plan.n_steps++;
    }
    int fin = -1;
    for (size_t t = 0; t < T.size(); ++t)
      if (T[t].alive) fin = int(t);
    TState& F = T[fin];
    // final tensor: rows = groups, dense = open legs
    std::set<int32_t> want;
    for (auto q : net.open) want.insert(net.out_label[q]);
    std::set<int32_t> have(F.dense.begin(), F.dense.end());
    if (want != have) fail(TNC_E_INVALID, "the contracted network does not end on the open legs");
    std::vector<int32_t> row_of(net.closed.size());
    for (size_t g = 0; g < net.closed.size(); ++g) {
      const uint64_t k = net.closed[g] & F.q;
      auto it = std::lower_bound(F.keys.begin(), F.keys.end(), k);
      row_of[g] = int32_t(it - F.keys.begin());
    }
    plan.row_of_off = add_const(row_of.data(), row_of.size() * 4);
    SliceSumArgs& s = plan.ss;
    s.L = int64_t(net.closed.size());
    s.n_open = int(net.open.size());
    s.f_row_stride = int64_t(1) << F.dense.size();
    s.f_slice_stride = sstride(F.buf);
    for (int t = 0; t < s.n_open; ++t)
      s.open_stride[t] = int64_t(1) << pos_of(F.dense, net.out_label[net.open[t]]);
    plan.final_buf = F.buf;
    Launch L;
    L.kind = K_SUM;
    L.inv = false;
    L.b_in0 = F.buf;
    L.rec_in0 = F.rec;
    L.bufs = {F.buf};
    L.info = tnc_step_info{K_SUM, 0, s.L, int64_t(1) << s.n_open, 0, 0, 0.0,
                           double(s.L << s.n_open) * (8.0 + 32.0)};
    plan.dep.push_back(L);
    // constants for slices, sampling
    plan.slice_ids_off = add_const(net.slice_ids.data(), net.slice_ids.size() * 8);
    plan.closed_off = add_const(net.closed.data(), net.closed.size() * 8);
    std::vector<int32_t> open_pad = net.open;
    open_pad.push_back(0);
    plan.open_off = add_const(open_pad.data(), open_pad.size() * 4);
    if (!plan.sl_table.empty()) {
      plan.sl_prefix_off = add_const(plan.sl_prefix.data(), plan.sl_prefix.size() * 8);
      // table is written after packing (destination offsets); reserve it now
      plan.sl_table_off = add_const(plan.sl_table.data(), plan.sl_table.size() * sizeof(SliceLeafEntry));
    }
    plan.b_norm = new_buf(uint64_t(plan.norm_parts + 1) * 8);
    const int64_t l = int64_t(1) << net.open.size();
    plan.b_cum = new_buf(uint64_t(l) * 8);
    plan.b_totals = new_buf(uint64_t(plan.L) * 8);
    plan.sample_chunk = std::max<int64_t>(plan.L, 65536);
    plan.b_samples = new_buf(uint64_t(plan.sample_chunk) * 8);
    plan.b_counter = new_buf(8);
    finish_records();
  }
};

void pack(tnc_plan_s& plan) {
  // lifetimes: phase-1 launches occupy [0, P), phase-2 launches [P, P + D)
  const int P = int(plan.inv.size()), D = int(plan.dep.size());
  const int END = P + D;
  auto touch = [&](int b, int t) {
    Buf& x = plan.bufs[b];
    x.t0 = std::min(x.t0, t);
    x.t1 = std::max(x.t1, t);
  };
  for (int i = 0; i < P; ++i)
    for (int b : plan.inv[i].bufs) touch(b, i);
  for (int i = 0; i < D; ++i)
    for (int b : plan.dep[i].bufs) touch(b, P + i);
  for (auto& b : plan.bufs) {
    if (b.is_const) continue;
    if (b.t1 < 0) { b.t0 = 0; b.t1 = END; }          // scratch kept for the whole call
    if (b.t0 < P && b.t1 >= P) b.to_end = true;       // invariant result read by slices
    if (b.to_end) b.t1 = END;
  }
  plan.consts_bytes = align_up(plan.consts.size());
  std::vector<int> order;
  for (size_t i = 0; i < plan.bufs.size(); ++i)
    if (!plan.bufs[i].is_const) order.push_back(int(i));
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    return plan.bufs[a].bytes != plan.bufs[b].bytes ? plan.bufs[a].bytes > plan.bufs[b].bytes : a < b;
  });
  std::vector<int> placed;
  uint64_t top = 0;
  for (int id : order) {
    Buf& b = plan.bufs[id];
    std::vector<std::pair<uint64_t, uint64_t>> busy;
    for (int o : placed) {
      const Buf& c = plan.bufs[o];
      if (c.t1 < b.t0 || b.t1 < c.t0) continue;
      busy.push_back({c.off, c.off + c.bytes});
    }
    std::sort(busy.begin(), busy.end());
    uint64_t at = 0;
    for (auto& iv : busy) {
      if (at + b.bytes <= iv.first) break;
      at = std::max(at, iv.second);
    }
    b.off = at;
    top = std::max(top, at + b.bytes);
    placed.push_back(id);
  }
  for (int id : order) plan.bufs[id].off += plan.consts_bytes;
  plan.ws_bytes = plan.consts_bytes + align_up(top);
  // the slice-leaf table holds workspace destinations
  for (auto& e : plan.sl_table) e.dst_off = int64_t(plan.bufs[e.dst_off].off / 8);
  if (!plan.sl_table.empty())
    std::memcpy(plan.consts.data() + plan.sl_table_off, plan.sl_table.data(),
                plan.sl_table.size() * sizeof(SliceLeafEntry));
}

// ------------------------------------------------------------------------------------
// execution

// Slices [pos, pos + n) of the list form batches of at most p.batch consecutive ids whose
// bits outside p.vary agree, so that the once-per-batch steps are right for every slice.
int64_t run_length(const tnc_plan_s& p, int64_t pos, int64_t n) {
  const int64_t nb = std::min<int64_t>(p.batch, n);
  const uint64_t* id = p.slice_ids.data() + 2 * pos;
  for (int64_t i = 1; i < nb; ++i)
    if (((id[2 * i] ^ id[0]) & ~p.vary[0]) || ((id[2 * i + 1] ^ id[1]) & ~p.vary[1])) return i;
  return nb;
}

// Algorithmic flops that contracting slices [first, first + count) executes.
double plan_work(const tnc_plan_s& p, int64_t first, int64_t count) {
  if (count <= 0) return 0.0;
  double f = p.flops_inv;
  for (int64_t pos = 0; pos < count;) {
    const int64_t nb = run_length(p, first + pos, count - pos);
    f += (p.flops_slice - p.flops_shared) * double(nb) + p.flops_shared;
    pos += nb;
  }
  return f;
}

struct Exec {
  tnc_plan_s& p;
  uint8_t* ws;
  hipStream_t s;
  // fault injection (servers created with TNC_FAULT=launch:N): launches left before the one
  // that fails; null when off
  int64_t* fault = nullptr;

  // one launch unit (a batch of slice steps, eager or a graph replay, or the invariant phase)
  // is about to be enqueued: the injected fault makes it fail before anything is enqueued
  void tick() {
    if (fault && *fault > 0 && --*fault == 0)
      fail(TNC_E_HIP, "injected launch failure (TNC_FAULT)");
  }
  float2* ptr(int b) const { return reinterpret_cast<float2*>(ws + p.bufs[b].off); }
  const int32_t* gat(int64_t off) const {
    return off < 0 ? nullptr : reinterpret_cast<const int32_t*>(ws + off);
  }

  hipEvent_t ev() {
    if (p.ev_used == p.ev_pool.size()) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      p.ev_pool.push_back(e);
    }
    return p.ev_pool[p.ev_used++];
  }

  int64_t plan_copies(const Launch& L, int64_t nb) const {
    return p.bufs[L.b_out].per_slice ? nb : 1;
  }

  int64_t* counter() const { return reinterpret_cast<int64_t*>(ws + p.bufs[p.b_counter].off); }

  // scale record r (copy 0) and its step in words per slice copy
  uint32_t* rec(int r) const {
    if (r < 0) return nullptr;
    const Rec& x = p.recs[size_t(r)];
    return reinterpret_cast<uint32_t*>(ws + p.bufs[p.rec_buf[x.block]].off) + x.index * kRecWords;
  }
  int64_t rec_step(int r) const {
    if (r < 0) return 0;
    const Rec& x = p.recs[size_t(r)];
    return x.per_slice ? p.rec_count[x.block] * kRecWords : 0;
  }

  void check(hipError_t err) {
    if (err != hipSuccess) fail(TNC_E_HIP, std::string("kernel launch: ") + hipGetErrorString(err));
  }

  // one launch of the program for nb slices (nb = 1 for the invariant phase)
  void launch(const Launch& L, int64_t nb_batch, double* amps, hipStream_t st, bool timed) {
    if (!L.enabled) return;
    const int64_t nb = L.shared ? 1 : nb_batch;   // a shared step runs for one copy
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
      e0 = ev();
      e1 = ev();
      HIPCHK(hipEventRecord(e0, st));
    }
    hipError_t err = hipSuccess;
    switch (L.kind) {
      case K_STREAM: {
        StreamArgs a = L.st;
        a.X = ptr(L.b_in0);
        a.S = ptr(L.b_in1);
        a.C = ptr(L.b_out);
        a.gx = gat(L.g0);
        a.gs = gat(L.g1);
        a.nb = nb;
        a.rec_x = rec(L.rec_in0);
        a.rec_s = rec(L.rec_in1);
        a.rec_c = rec(L.rec_out);
        a.rec_x_step = rec_step(L.rec_in0);
        a.rec_s_step = rec_step(L.rec_in1);
        a.rec_c_step = rec_step(L.rec_out);
        err = launch_stream(a, st);
        break;
      }
      case K_GEMM: {
        GemmArgs a = L.gm;
        a.A = ptr(L.b_in0);
        a.B = ptr(L.b_in1);
        a.C = ptr(L.b_out);
        a.ga = gat(L.g0);
        a.gb = gat(L.g1);
        a.stk = gat(L.stk_off);
        a.perm = gat(L.perm_off);
        a.rec_a = rec(L.rec_in0);
        a.rec_b = rec(L.rec_in1);
        a.rec_c = rec(L.rec_out);
        a.rec_a_step = rec_step(L.rec_in0);
        a.rec_b_step = rec_step(L.rec_in1);
        a.rec_c_step = rec_step(L.rec_out);
        a.partial = L.b_tmp >= 0 ? ptr(L.b_tmp) : nullptr;
        a.nb = nb;
        err = launch_gemm(a, st);
        break;
      }
      case K_SPLIT: {
        const int64_t copies = plan_copies(L, nb);
        err = launch_zero_u32(reinterpret_cast<uint32_t*>(ptr(L.b_out)), copies * L.n_elems, st);
        break;
      }
      case K_REDUCE: {
        ReduceArgs a = L.rd;
        a.partial = ptr(L.b_in0);
        a.C = ptr(L.b_out);
        a.elems = L.rd.elems * nb;
        a.rec = rec(L.rec_out);
        a.rec_step = rec_step(L.rec_out);
        err = launch_reduce(a, st);
        break;
      }
      case K_LEAVES: {
        SliceLeafArgs a{};
        a.table = reinterpret_cast<const SliceLeafEntry*>(ws + p.sl_table_off);
        a.prefix = reinterpret_cast<const int64_t*>(ws + p.sl_prefix_off);
        a.n_entries = int(p.sl_table.size());
        a.consts = reinterpret_cast<const float2*>(ws);
        a.ws = reinterpret_cast<float2*>(ws);
        a.slice_ids = reinterpret_cast<const uint64_t*>(ws + p.slice_ids_off);
        a.base = counter();
        a.nb = nb;
        err = launch_slice_leaves(a, p.sl_total, st);
        break;
      }
      case K_SUM: {
        SliceSumArgs a = p.ss;
        a.F = ptr(L.b_in0);
        a.amps = amps;
        a.row_of = reinterpret_cast<const int32_t*>(ws + p.row_of_off);
        a.overwrite = 0;
        a.nb = nb;
        a.rec_f = rec(L.rec_in0);
        a.rec_f_step = rec_step(L.rec_in0);
        err = launch_slice_sum(a, st);
        break;
      }
    }
    check(err);
    if (timed) {
      HIPCHK(hipEventRecord(e1, st));
      int index = -1;
      if (!p.inv.empty() && &L >= p.inv.data() && &L < p.inv.data() + p.inv.size())
        index = int(&L - p.inv.data());
      else if (!p.dep.empty() && &L >= p.dep.data() && &L < p.dep.data() + p.dep.size())
        index = int(p.inv.size()) + int(&L - p.dep.data());
      p.pending.push_back(
          TimingRec{L.kind, index, L.info.bytes * double(nb), L.info.flops * double(nb), e0, e1});
    }
  }

  // the per-batch program: every slice-dependent launch, then the slice counter advance
  void batch(int64_t nb, double* amps, hipStream_t st, bool timed) {
    for (auto& L : p.dep) launch(L, nb, amps, st, timed);
    check(launch_add_i64(counter(), nb, st));
  }

  void capture(double* amps) {
    if (p.graph && p.graph_ws == ws && p.graph_amps == amps) return;
    if (p.graph) {
      HIPCHK(hipGraphExecDestroy(p.graph));
      p.graph = nullptr;
    }
    if (!p.capture_stream) HIPCHK(hipStreamCreateWithFlags(&p.capture_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(p.capture_stream, hipStreamCaptureModeThreadLocal));
    try {
      batch(p.batch, amps, p.capture_stream, false);
    } catch (...) {
      (void)hipStreamEndCapture(p.capture_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HIPCHK(hipStreamEndCapture(p.capture_stream, &g));
    hipError_t e = hipGraphInstantiate(&p.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) fail(TNC_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    p.graph_ws = ws;
    p.graph_amps = amps;
  }

  void upload() {
    if (p.uploaded_ws == ws) return;
    HIPCHK(hipMemcpyAsync(ws, p.consts.data(), p.consts.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    p.uploaded_ws = ws;
  }

  // skip_invariant: the slice-invariant results already sit in this workspace from an
  // earlier call with the same workspace (their buffers are never reused by slice steps)
  void contract(double* amps, int64_t first, int64_t count, bool accumulate,
                bool skip_invariant = false) {
    upload();
    const int64_t n_amp = p.L << p.n_open;
    if (!accumulate) check(launch_fill_zero(amps, 2 * n_amp, s));
    if (count <= 0) return;
    if (!skip_invariant) {
      tick();
      for (auto& L : p.inv) launch(L, 1, amps, s, p.timing);
    }
    check(launch_set_i64(counter(), first, s));
    const int64_t S = p.batch;
    static const bool no_graph = std::getenv("TNC_NO_GRAPH") != nullptr;
    // Full batches replay the captured graph.  With timing on, a bounded sample of batches
    // (about 4096 launches per call) is launched eagerly with an event pair per launch.
    const int64_t nbat = (count + S - 1) / S;
    int64_t stride = nbat + 1;
    if (p.timing) {
      const int64_t per = std::max<int64_t>(1, int64_t(p.dep.size()));
      const int64_t n_timed = std::max<int64_t>(1, 4096 / per);
      stride = std::max<int64_t>(1, nbat / n_timed);
    }
    bool captured = false;
    for (int64_t pos = 0, b = 0; pos < count; ++b) {
      const int64_t nb = run_length(p, first + pos, count - pos);
      const bool timed = p.timing && (b % stride == 0);
      tick();
      if (timed || no_graph || nb < S) {
        batch(nb, amps, s, timed);
      } else {
        if (!captured) capture(amps);
        captured = true;
        HIPCHK(hipGraphLaunch(p.graph, s));
      }
      pos += nb;
    }
  }
};

void harvest(tnc_plan_s& p) {
  for (auto& r : p.pending) {
    HIPCHK(hipEventSynchronize(r.e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, r.e0, r.e1));
    p.t_ms[r.kind] += ms;
    p.t_bytes[r.kind] += r.bytes;
    p.t_flops[r.kind] += r.flops;
    p.t_n[r.kind] += 1;
    if (r.index >= 0) {
      const size_t n = p.inv.size() + p.dep.size();
      if (p.l_ms.size() != n) {
        p.l_ms.assign(n, 0.0);
        p.l_n.assign(n, 0);
      }
      p.l_ms[size_t(r.index)] += ms;
      p.l_n[size_t(r.index)] += 1;
    }
  }
  p.pending.clear();
  p.ev_used = 0;
}

// Launch the draws [done, done + c) of tnc_sample into the plan's sample buffer on `st`
// (asynchronous) and return c; *d_out receives the buffer.  With several groups all L draws
// are launched at once (done = 0); with one group at most sample_chunk, and the draw index
// keeps counting across chunks.
int64_t launch_draws(tnc_plan_s& p, uint8_t* ws, const double* amps, uint64_t seed, int64_t done,
                     int64_t n_samples, hipStream_t st, const uint64_t** d_out) {
  double* cum = reinterpret_cast<double*>(ws + p.bufs[p.b_cum].off);
  uint64_t* dout = reinterpret_cast<uint64_t*>(ws + p.bufs[p.b_samples].off);
  const uint64_t* closed = reinterpret_cast<const uint64_t*>(ws + p.closed_off);
  const int32_t* openq = reinterpret_cast<const int32_t*>(ws + p.open_off);
  *d_out = dout;
  int64_t c = p.L;
  hipError_t err;
  if (p.L > 1) {
    err = launch_sample(amps, p.L, p.n_open, closed, openq, p.n_qubits, seed, p.L, cum, dout, st);
  } else {
    c = std::min(p.sample_chunk, n_samples - done);
    // shift the counter: uniform j uses state seed + (j + 1) gamma
    const uint64_t seed_c = seed + uint64_t(done) * 0x9E3779B97F4A7C15ull;
    err = launch_sample(amps, 1, p.n_open, closed, openq, p.n_qubits, seed_c, c, cum, dout, st);
  }
  if (err != hipSuccess) fail(TNC_E_HIP, hipGetErrorString(err));
  return c;
}

// Draws of tnc_sample; synchronous on `st`.
void sample_into(tnc_plan_s& p, uint8_t* ws, const double* amps, uint64_t seed, int64_t n_samples,
                 uint64_t* h_bits, hipStream_t st) {
  if (n_samples < 0) fail(TNC_E_INVALID, "negative sample count");
  if (p.L > 1 && n_samples != p.L)
    fail(TNC_E_INVALID, "with several groups, n_samples must equal the number of groups");
  Exec e{p, ws, st};
  e.upload();
  for (int64_t done = 0; done < n_samples;) {
    const uint64_t* dout = nullptr;
    const int64_t c = launch_draws(p, ws, amps, seed, done, n_samples, st, &dout);
    HIPCHK(hipMemcpyAsync(h_bits + done, dout, uint64_t(c) * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    done += c;
  }
}

// In-group Metropolis chains (steps >= 0) or frugal rejection sampling (trials >= 1, m > 0);
// synchronous on `st`.  Draw d keeps counting across chunks of one group's draws.
void sample_chain_into(tnc_plan_s& p, uint8_t* ws, const double* amps, uint64_t seed,
                       int64_t n_samples, bool frugal, int32_t steps_or_trials, double m,
                       uint64_t* h_bits, hipStream_t st) {
  if (n_samples < 0) fail(TNC_E_INVALID, "negative sample count");
  if (p.L > 1 && n_samples != p.L)
    fail(TNC_E_INVALID, "with several groups, n_samples must equal the number of groups");
  if (frugal && (steps_or_trials < 1 || !(m > 0.0) || !std::isfinite(m)))
    fail(TNC_E_INVALID, "frugal sampling needs trials >= 1 and a finite m > 0");
  if (!frugal && steps_or_trials < 0) fail(TNC_E_INVALID, "negative chain length");
  Exec e{p, ws, st};
  e.upload();
  uint64_t* dout = reinterpret_cast<uint64_t*>(ws + p.bufs[p.b_samples].off);
  double* totals = reinterpret_cast<double*>(ws + p.bufs[p.b_totals].off);
  const uint64_t* closed = reinterpret_cast<const uint64_t*>(ws + p.closed_off);
  const int32_t* openq = reinterpret_cast<const int32_t*>(ws + p.open_off);
  if (frugal && n_samples > 0) e.check(launch_group_totals(amps, p.L, p.n_open, totals, st));
  for (int64_t done = 0; done < n_samples; done += p.sample_chunk) {
    const int64_t c = std::min(p.sample_chunk, n_samples - done);
    e.check(frugal ? launch_sample_frugal(amps, totals, p.L, p.n_open, closed, openq, p.n_qubits,
                                          seed, done, c, m, steps_or_trials, dout, st)
                   : launch_sample_metropolis(amps, p.L, p.n_open, closed, openq, p.n_qubits,
                                              seed, done, c, steps_or_trials, dout, st));
    HIPCHK(hipMemcpyAsync(h_bits + done, dout, uint64_t(c) * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
}

tnc_plan_s* compile_plan(tnc_net_s& net, tnc_precision precision, int32_t max_batch);

// TNC_PLAN_LOG: one line per GEMM launch (shape, tiles, split-K, row folding or stacking)
void log_plan(const tnc_plan_s& p) {
  for (int phase = 0; phase < 2; ++phase)
    for (const Launch& L : phase == 0 ? p.inv : p.dep) {
      if (L.kind == K_STREAM) {
        const StreamArgs& a = L.st;
        std::string kins, spos;
        for (int j = 0; j < a.nk; ++j) kins += " " + std::to_string(a.x_kins[j]);
        for (int j = 0; j < a.nk; ++j) spos += " k" + std::to_string(a.s_kpos[j]);
        for (int j = 0; j < a.nn; ++j) spos += " n" + std::to_string(a.s_npos[j]);
        std::fprintf(stderr,
                     "[tnc plan] %s stream rows %lld x_rows %lld s_rows %lld | m 2^%d k 2^%d n 2^%d | "
                     "x k-bits at%s | s bits%s | gx %d gs %d\n",
                     phase == 0 ? "inv" : "dep", (long long)a.rows, (long long)a.x_rows,
                     (long long)a.s_rows, a.n_m, a.nk, a.nn, kins.c_str(), spos.c_str(),
                     L.g0 >= 0 ? 1 : 0, L.g1 >= 0 ? 1 : 0);
        continue;
      }
      if (L.kind != K_GEMM) continue;
      const GemmArgs& g = L.gm;
      // bit positions of the m, k (A) and k, n (B) indices in the operands' dense index
      std::string pos = " | A m";
      for (int j = 0; j < g.nm; ++j) pos += " " + std::to_string(g.a_mpos[j]);
      pos += " k";
      for (int j = 0; j < g.nk; ++j) pos += " " + std::to_string(g.a_kpos[j]);
      pos += " | B k";
      for (int j = 0; j < g.nk; ++j) pos += " " + std::to_string(g.b_kpos[j]);
      pos += " n";
      for (int j = 0; j < g.nn; ++j) pos += " " + std::to_string(g.b_npos[j]);
      std::fprintf(stderr,
                   "[tnc plan] %s gemm rows %lld M %lld N %lld K %lld | launch M %lld rows %lld "
                   "config %d splits %d fold %d stacked %d | a_rows %lld b_rows %lld | %.3g GF%s\n",
                   phase == 0 ? "inv" : "dep", (long long)L.info.rows, (long long)L.info.m,
                   (long long)L.info.n, (long long)L.info.k, (long long)g.M, (long long)g.rows,
                   g.config, g.k_splits, g.fold, L.stk_off >= 0 ? 1 : 0, (long long)g.a_rows,
                   (long long)g.b_rows, L.info.flops / 1e9, pos.c_str());
    }
}

// Automatic batch size: the smallest power of two whose batch carries at least
// kAutoBatchFlops of dependent work (so launch latency stays small against it), capped at
// kAutoBatchMax, at the slice count, and at what fits `budget` bytes of workspace.
constexpr double kAutoBatchFlops = 2.5e11;
constexpr int32_t kAutoBatchMax = 256;

tnc_plan_s* make_plan(tnc_net_s& net, tnc_precision precision, int32_t max_batch,
                      uint64_t budget = uint64_t(16) << 30) {
  if (max_batch < 0) fail(TNC_E_INVALID, "max_batch_slices must be >= 0 (0 = automatic)");
  if (max_batch > 0) return compile_plan(net, precision, max_batch);
  tnc_plan_s* one = compile_plan(net, precision, 1);
  const int64_t n = one->n_slices();
  if (n <= 1) return one;
  const uint64_t ws1 = one->ws_bytes;
  const double f = std::max(1.0, one->flops_slice);
  delete one;
  tnc_plan_s* two = compile_plan(net, precision, 2);
  const uint64_t per = two->ws_bytes > ws1 ? two->ws_bytes - ws1 : 1;
  delete two;
  int32_t S = 1;
  while (S < kAutoBatchMax && S < n && double(S) * f < kAutoBatchFlops &&
         ws1 + uint64_t(2 * S - 1) * per <= budget)
    S *= 2;
  return compile_plan(net, precision, S);
}

tnc_plan_s* compile_plan(tnc_net_s& net, tnc_precision precision, int32_t max_batch) {
  if (!net.has_path && net.labels.size() > 1) fail(TNC_E_INVALID, "no path set");
  if (!net.has_targets) fail(TNC_E_INVALID, "no targets set");
  if (precision != TNC_C64 && precision != TNC_BF16X3 && precision != TNC_FP16X3)
    fail(TNC_E_UNSUPPORTED, "implemented precisions: TNC_C64, TNC_BF16X3, TNC_FP16X3");
  if (max_batch < 1) fail(TNC_E_INVALID, "max_batch_slices must be >= 1");
  auto* p = new tnc_plan_s();
  try {
    p->device = net.device;
    p->n_qubits = net.n_qubits;
    p->precision = precision;
    p->L = int64_t(net.closed.size());
    p->n_open = int(net.open.size());
    p->open = net.open;
    p->closed = net.closed;
    p->slice_ids = net.slice_ids;
    p->batch = std::max<int32_t>(
        1, int32_t(std::min<int64_t>(max_batch, int64_t(net.slice_ids.size() / 2))));
    // bits that vary inside the batches of a full pass; TNC_NO_SHARE turns sharing off
    if (std::getenv("TNC_NO_SHARE") == nullptr) {
      p->vary[0] = p->vary[1] = 0;
      const int64_t n = p->n_slices();
      const uint64_t* id = p->slice_ids.data();
      for (int64_t b0 = 0; b0 < n; b0 += p->batch)
        for (int64_t i = b0 + 1; i < std::min<int64_t>(n, b0 + p->batch); ++i) {
          p->vary[0] |= id[2 * i] ^ id[2 * b0];
          p->vary[1] |= id[2 * i + 1] ^ id[2 * b0 + 1];
        }
    }
    Compiler c(net, *p);
    c.run();
    pack(*p);
    if (std::getenv("TNC_PLAN_LOG")) log_plan(*p);
  } catch (...) {
    delete p;
    throw;
  }
  return p;
}

// ------------------------------------------------------------------------------------
// autotuner: per GEMM launch, time the tile configurations (and split-K factors up to the
// one its partial buffer was sized for) on the real workspace and keep the fastest.
// Results are cached per shape for the process and, when TNC_TUNE_CACHE names a file,
// across processes (one "key config splits" line per shape).
std::mutex g_tune_mu;
std::map<std::string, std::pair<int, int>> g_tune;
bool g_tune_loaded = false;

std::string tune_key(const GemmArgs& g, int64_t nb) {
  return std::to_string(g.M) + "x" + std::to_string(g.N) + "x" + std::to_string(g.K) + "/r" +
         std::to_string(g.rows) + "/b" + std::to_string(nb) + "/f" + std::to_string(g.a_mfast) +
         std::to_string(g.b_nfast) + "/p" + std::to_string(g.precision) + "/g" +
         std::to_string(g.ga != nullptr || g.gb != nullptr) + "/s" + std::to_string(g.stk != nullptr);
}

void tune_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("TNC_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char key[256];
  int c, sp;
  while (std::fscanf(f, "%255s %d %d", key, &c, &sp) == 3) g_tune[key] = {c, sp};
  std::fclose(f);
}

void tune_store(const std::string& key, int c, int sp) {
  g_tune[key] = {c, sp};
  const char* path = std::getenv("TNC_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d\n", key.c_str(), c, sp);
  std::fclose(f);
}

int autotune(tnc_plan_s& p, uint8_t* ws, hipStream_t st, int reps) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load();
  Exec e{p, ws, st};
  e.upload();
  e.check(launch_set_i64(e.counter(), 0, st));
  // cleared scale records: the timed launches read defined (zero) largest components
  for (int phase = 0; phase < 2; ++phase)
    for (const Launch& L : phase == 0 ? p.inv : p.dep)
      if (L.kind == K_SPLIT) e.launch(L, phase == 0 ? 1 : p.batch, nullptr, st, false);
  int changed = 0;
  hipEvent_t t0, t1;
  HIPCHK(hipEventCreate(&t0));
  HIPCHK(hipEventCreate(&t1));
  for (int phase = 0; phase < 2; ++phase) {
    std::vector<Launch>& lst = phase == 0 ? p.inv : p.dep;
    for (size_t i = 0; i < lst.size(); ++i) {
      Launch& L = lst[i];
      if (L.kind != K_GEMM) continue;
      const int64_t nb = (phase == 0 || L.shared) ? 1 : p.batch;
      Launch* R = (i + 1 < lst.size() && lst[i + 1].kind == K_REDUCE && lst[i + 1].b_in0 == L.b_tmp)
                      ? &lst[i + 1] : nullptr;
      GemmArgs probe = L.gm;
      probe.ga = e.gat(L.g0);
      probe.gb = e.gat(L.g1);
      probe.stk = e.gat(L.stk_off);
      const std::string key = tune_key(probe, nb);
      std::pair<int, int> best{L.gm.config, L.gm.k_splits};
      auto hit = g_tune.find(key);
      if (hit != g_tune.end() && hit->second.second <= L.max_splits) {
        best = hit->second;
      } else {
        // the planned choice is timed first, so that it survives ties
        std::vector<std::pair<int, int>> cands{best};
        GemmArgs one = L.gm;
        one.k_splits = 1;
        const bool narrow = gemm_rows_narrow_fits(one, L.stk_off >= 0);
        for (int cfg = 0; cfg < Compiler::kConfigs; ++cfg) {
          if (cfg == 5 && L.gm.precision != 0 && !narrow) continue;
          if (cfg == 6 && !Compiler::outer_ok(L.gm, L.stk_off >= 0)) continue;
          if (cfg >= 7 && !Compiler::big_ok(L.gm, L.stk_off >= 0)) continue;
          for (int sp = 1; sp <= (cfg == 6 ? 1 : L.max_splits); sp *= 2)
            if ((sp == 1 || L.gm.K / sp >= 256) && std::make_pair(cfg, sp) != best)
              cands.push_back({cfg, sp});
        }
        float best_ms = 1e30f;
        for (const auto& cand : cands) {
          {
            const int cfg = cand.first, sp = cand.second;
            Launch G = L;
            G.gm.config = cfg;
            G.gm.k_splits = sp;
            G.gm.k_chunk = L.gm.K / sp;
            float total = 0;
            for (int r = 0; r <= reps; ++r) {   // the first run warms caches, not counted
              HIPCHK(hipEventRecord(t0, st));
              e.launch(G, nb, nullptr, st, false);
              if (sp > 1 && R) {
                Launch Rr = *R;
                Rr.enabled = true;
                Rr.rd.splits = sp;
                e.launch(Rr, nb, nullptr, st, false);
              }
              HIPCHK(hipEventRecord(t1, st));
              HIPCHK(hipEventSynchronize(t1));
              float ms = 0;
              HIPCHK(hipEventElapsedTime(&ms, t0, t1));
              if (r > 0) total += ms;
            }
            if (total < best_ms * 0.98f) {   // within 2%: keep the earlier choice
              best_ms = total;
              best = cand;
            }
          }
        }
        tune_store(key, best.first, best.second);
      }
      if (best.first != L.gm.config || best.second != L.gm.k_splits) ++changed;
      L.gm.config = best.first;
      L.gm.k_splits = best.second;
      L.gm.k_chunk = L.gm.K / best.second;
      if (R) {
        R->enabled = best.second > 1;
        R->rd.splits = best.second;
      }
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (p.graph) {
    HIPCHK(hipGraphExecDestroy(p.graph));
    p.graph = nullptr;
  }
  return changed;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    HIPCHK(hipGetDevice(&prev));
    if (prev != dev) HIPCHK(hipSetDevice(dev));
  }
  ~DeviceGuard() {
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace


// ------------------------------------------------------------------------------------
// serving: continuous batching of contraction requests on one device
namespace {

enum ReqState { R_QUEUED, R_RUNNING, R_DONE, R_FAILED };

struct Request {
  uint64_t id = 0;
  tnc_plan_s* plan = nullptr;
  int64_t n_samples = 0;
  uint64_t seed = 0;
  uint64_t ws_bytes = 0, amps_bytes = 0, footprint = 0, off = 0;
  int slot = -1;
  int64_t next = 0, total = 0;
  std::deque<hipEvent_t> chunks;        // chunks in flight, oldest first
  // end of the request: amplitudes and draws copied to the slot's pinned staging, polled
  // through `fin` (draws in chunks of the plan's sample_chunk with one group)
  bool finishing = false, amps_taken = false;
  int64_t drawn = 0, last_draws = 0;
  hipEvent_t fin = nullptr;
  ReqState state = R_QUEUED;
  std::vector<double> amps;
  std::vector<uint64_t> bits;
  double norm = 0, t_submit = 0, t_admit = 0, t_done = 0;
  tnc_status code = TNC_OK;
  std::string err;
  ~Request() { delete plan; }
};

}  // namespace

struct tnc_server_s {
  int device = 0;
  uint8_t* arena = nullptr;
  uint64_t arena_bytes = 0;
  int max_slots = 1;
  int chunk_batches = 4;
  std::map<uint64_t, uint64_t> free_list;     // arena offset -> bytes
  std::vector<hipStream_t> streams;
  std::vector<bool> slot_busy;
  std::vector<hipEvent_t> ev_free;
  std::vector<uint8_t*> pin;                  // per slot: pinned host staging of results
  std::vector<uint64_t> pin_cap;
  int64_t fault_left = 0;                     // TNC_FAULT=launch:N (worker thread only)
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> pending;
  std::vector<Request*> active;
  std::map<uint64_t, Request*> all;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread worker;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  bool alloc(uint64_t bytes, uint64_t* off) {
    for (auto it = free_list.begin(); it != free_list.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const uint64_t rest = it->second - bytes, at = it->first + bytes;
      free_list.erase(it);
      if (rest) free_list[at] = rest;
      return true;
    }
    return false;
  }

  void release(uint64_t off, uint64_t bytes) {
    auto it = free_list.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_list.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_list.erase(nx);
    }
    if (it != free_list.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_list.erase(it);
      }
    }
  }

  hipEvent_t get_event() {
    if (!ev_free.empty()) {
      hipEvent_t e = ev_free.back();
      ev_free.pop_back();
      return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return e;
  }

  // pinned host staging of slot k, at least `bytes` (its earlier copies have completed)
  uint8_t* staging(int k, uint64_t bytes) {
    if (pin_cap[size_t(k)] < bytes) {
      if (pin[size_t(k)]) HIPCHK(hipHostFree(pin[size_t(k)]));
      pin[size_t(k)] = nullptr;
      pin_cap[size_t(k)] = 0;
      HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&pin[size_t(k)]), bytes, hipHostMallocDefault));
      pin_cap[size_t(k)] = bytes;
    }
    return pin[size_t(k)];
  }

  uint64_t amp_bytes(const Request& r) const { return uint64_t(r.plan->L << r.plan->n_open) * 16; }

  // enqueue the amplitudes' copy (first time) and the next chunk of draws with its copy, all
  // into the slot's staging, and mark their completion with r.fin; nothing waits here
  void enqueue_finish(Request& r, const double* amps, hipStream_t st) {
    const int64_t per = r.plan->L > 1 ? r.plan->L : std::min(r.plan->sample_chunk, r.n_samples);
    const uint64_t ab = amp_bytes(r), off_bits = align_up(ab);
    uint8_t* h = staging(r.slot, off_bits + uint64_t(std::max<int64_t>(per, 0)) * 8);
    if (!r.amps_taken) HIPCHK(hipMemcpyAsync(h, amps, ab, hipMemcpyDeviceToHost, st));
    r.last_draws = 0;
    if (r.drawn < r.n_samples) {
      const uint64_t* dout = nullptr;
      r.last_draws = launch_draws(*r.plan, arena + r.off, amps, r.seed, r.drawn, r.n_samples, st,
                                  &dout);
      HIPCHK(hipMemcpyAsync(h + off_bits, dout, uint64_t(r.last_draws) * 8,
                            hipMemcpyDeviceToHost, st));
    }
    if (!r.fin) r.fin = get_event();
    HIPCHK(hipEventRecord(r.fin, st));
    r.finishing = true;
  }

  // enqueue the next chunk of slices; once every chunk has completed, the end of the request
  // (draws and copies) is enqueued and polled like the chunks: the worker never waits on a
  // request's stream, so other requests keep being fed meanwhile
  bool step(Request& r) {
    uint8_t* ws = arena + r.off;
    double* amps = reinterpret_cast<double*>(ws + align_up(r.ws_bytes));
    hipStream_t st = streams[size_t(r.slot)];
    if (r.finishing) {
      const hipError_t q = hipEventQuery(r.fin);
      if (q == hipErrorNotReady) return false;
      if (q != hipSuccess) fail(TNC_E_HIP, std::string("request end: ") + hipGetErrorString(q));
      const uint8_t* h = pin[size_t(r.slot)];
      if (!r.amps_taken) {
        r.amps.resize(amp_bytes(r) / 8);
        std::memcpy(r.amps.data(), h, amp_bytes(r));
        double nrm = 0;
        for (double x : r.amps) nrm += x * x;
        r.norm = nrm;
        r.amps_taken = true;
      }
      if (r.last_draws > 0) {
        std::memcpy(r.bits.data() + r.drawn, h + align_up(amp_bytes(r)), size_t(r.last_draws) * 8);
        r.drawn += r.last_draws;
      }
      if (r.drawn < r.n_samples) {
        enqueue_finish(r, amps, st);
      } else {
        r.finishing = false;
        r.state = R_DONE;
      }
      return true;
    }
    bool did = false;
    while (!r.chunks.empty() && hipEventQuery(r.chunks.front()) == hipSuccess) {
      ev_free.push_back(r.chunks.front());
      r.chunks.pop_front();
      did = true;
    }
    if (r.next < r.total && r.chunks.size() < 2) {
      const int64_t count = std::min<int64_t>(int64_t(chunk_batches) * r.plan->batch, r.total - r.next);
      Exec e{*r.plan, ws, st};
      if (fault_left > 0) e.fault = &fault_left;
      e.contract(amps, r.next, count, r.next > 0, r.next > 0);
      hipEvent_t ev = get_event();
      HIPCHK(hipEventRecord(ev, st));
      r.chunks.push_back(ev);
      r.next += count;
      did = true;
    }
    if (r.next >= r.total && r.chunks.empty()) {
      if (r.n_samples > 0) r.bits.resize(size_t(r.n_samples));
      enqueue_finish(r, amps, st);
      did = true;
    }
    return did;
  }

  void retire_from_active(Request* r) {
    // caller holds mu
    release(r->off, r->footprint);
    slot_busy[r->slot] = false;
    for (auto e : r->chunks) ev_free.push_back(e);
    r->chunks.clear();
    if (r->fin) ev_free.push_back(r->fin);
    r->fin = nullptr;
    r->finishing = false;
    r->t_done = now();
    active.erase(std::find(active.begin(), active.end(), r));
  }

  void run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      if (stop) break;
      // admission: first come first served, while a slot and a large enough block exist
      while (!pending.empty() && int(active.size()) < max_slots) {
        Request* r = pending.front();
        uint64_t off;
        if (!alloc(r->footprint, &off)) break;
        pending.pop_front();
        r->off = off;
        for (int k = 0; k < max_slots; ++k)
          if (!slot_busy[k]) { r->slot = k; slot_busy[k] = true; break; }
        r->state = R_RUNNING;
        r->t_admit = now();
        active.push_back(r);
      }
      if (active.empty()) {
        cv.wait(lk, [&] { return stop || !pending.empty(); });
        continue;
      }
      std::vector<Request*> act = active;
      lk.unlock();
      bool did = false;
      std::vector<Request*> finished;
      for (Request* r : act) {
        try {
          did |= step(*r);
        } catch (const Error& e) {
          r->state = R_FAILED;
          r->code = e.code;
          r->err = e.msg;
          (void)hipStreamSynchronize(streams[r->slot]);
        } catch (const std::exception& e) {
          r->state = R_FAILED;
          r->code = TNC_E_INTERNAL;
          r->err = e.what();
          (void)hipStreamSynchronize(streams[r->slot]);
        }
        if (r->state == R_DONE || r->state == R_FAILED) finished.push_back(r);
      }
      lk.lock();
      for (Request* r : finished) retire_from_active(r);
      if (!finished.empty()) cv.notify_all();
      if (!did && finished.empty()) {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(50));
        lk.lock();
      }
    }
    // shutting down: let queued device work finish before the arena goes away
    for (auto st : streams) (void)hipStreamSynchronize(st);
  }

  ~tnc_server_s() {
    {
      std::lock_guard<std::mutex> g(mu);
      stop = true;
    }
    cv.notify_all();
    if (worker.joinable()) worker.join();
    for (auto& kv : all) delete kv.second;
    for (auto e : ev_free) (void)hipEventDestroy(e);
    for (auto h : pin)
      if (h) (void)hipHostFree(h);
    for (auto st : streams) (void)hipStreamDestroy(st);
  }
};

// ------------------------------------------------------------------------------------
// C ABI
// ---- sampling out of a caller-given scratch buffer (used by tnc_sample_noalloc) ----
tnc_status tnc::report_error(tnc_status code, const char* msg) {
  g_err = msg ? msg : "";
  return code;
}

tnc_status tnc::plan_device(tnc_plan p, int* device) {
  return guard([&] {
    if (!p || !device) fail(TNC_E_INVALID, "null argument");
    *device = p->device;
  });
}

tnc_status tnc::sample_in_scratch(tnc_plan p, uint8_t* scratch, uint64_t cap, const double* amps,
                                  uint64_t seed, int64_t n_samples, uint64_t* h_bits,
                                  void* stream) {
  return guard([&] {
    if (!p || !scratch || !amps || (n_samples > 0 && !h_bits)) fail(TNC_E_INVALID, "null argument");
    if (n_samples < 0) fail(TNC_E_INVALID, "negative sample count");
    if (p->L > 1 && n_samples != p->L)
      fail(TNC_E_INVALID, "with several groups, n_samples must equal the number of groups");
    DeviceGuard dg(p->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint64_t L = uint64_t(p->L), l = uint64_t(1) << p->n_open;
    // layout: closed bits | open qubit ids | running sums (one group only) | draws
    const uint64_t o_open = align_up(L * 8), o_cum = o_open + align_up(4 * 64 + 4);
    const uint64_t o_out = o_cum + (L == 1 ? align_up(l * 8) : 0);
    const uint64_t need = o_out + 8 * (L > 1 ? L : 1);
    if (need > cap)
      fail(TNC_E_INVALID, "sampling this plan needs " + std::to_string(need) +
                              " bytes of scratch, more than the " + std::to_string(cap) +
                              " bytes of tnc_sample_noalloc's static buffer");
    HIPCHK(hipMemcpyAsync(scratch, p->consts.data() + p->closed_off, L * 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(scratch + o_open, p->consts.data() + p->open_off,
                          4 * uint64_t(p->n_open + 1), hipMemcpyHostToDevice, st));
    const uint64_t* closed = reinterpret_cast<const uint64_t*>(scratch);
    const int32_t* openq = reinterpret_cast<const int32_t*>(scratch + o_open);
    double* cum = reinterpret_cast<double*>(scratch + o_cum);
    uint64_t* dout = reinterpret_cast<uint64_t*>(scratch + o_out);
    if (n_samples == 0) {
      HIPCHK(hipStreamSynchronize(st));
      return;
    }
    // one group: the draws go out in chunks that fill the rest of the buffer (the draw
    // index keeps counting across chunks, as in tnc_sample); several groups: one launch
    const int64_t chunk = L > 1 ? int64_t(L) : int64_t((cap - o_out) / 8);
    for (int64_t done = 0; done < n_samples; done += chunk) {
      const int64_t c = std::min(chunk, n_samples - done);
      const uint64_t seed_c = L > 1 ? seed : seed + uint64_t(done) * 0x9E3779B97F4A7C15ull;
      hipError_t err = launch_sample(amps, p->L, p->n_open, closed, openq, p->n_qubits, seed_c, c,
                                     cum, dout, st);
      if (err != hipSuccess) fail(TNC_E_HIP, hipGetErrorString(err));
      HIPCHK(hipMemcpyAsync(h_bits + done, dout, uint64_t(c) * 8, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
    }
  });
}

extern "C" {

const char* tnc_last_error(void) { return g_err.c_str(); }

tnc_status tnc_net_create(int device, const tnc_network_desc* d, tnc_net* out) {
  return guard([&] {
    if (!d || !out) fail(TNC_E_INVALID, "null argument");
    *out = nullptr;
    if (d->n_qubits < 0 || d->n_qubits > 64) fail(TNC_E_INVALID, "n_qubits must be in [0, 64]");
    if (d->n_tensors < 1) fail(TNC_E_INVALID, "a network needs at least one tensor");
    if (!d->ranks || !d->labels || !d->data || (d->n_qubits > 0 && !d->out_label))
      fail(TNC_E_INVALID, "null array in the network description");
    auto* n = new tnc_net_s();
    try {
      n->device = device;
      n->n_qubits = d->n_qubits;
      int64_t lp = 0, dp = 0;
      for (int t = 0; t < d->n_tensors; ++t) {
        const int r = d->ranks[t];
        if (r < 0 || r > kMaxRank) fail(TNC_E_INVALID, "tensor rank out of range [0, 40]");
        std::vector<int32_t> lab(d->labels + lp, d->labels + lp + r);
        for (auto x : lab) {
          if (x < 0) fail(TNC_E_INVALID, "negative label");
          n->holders[x].push_back(t);
        }
        std::set<int32_t> uniq(lab.begin(), lab.end());
        if (int(uniq.size()) != r) fail(TNC_E_INVALID, "a tensor repeats a label");
        const int64_t sz = int64_t(1) << r;
        n->labels.push_back(lab);
        n->data.emplace_back(d->data + dp, d->data + dp + 2 * sz);
        lp += r;
        dp += 2 * sz;
      }
      for (auto& kv : n->holders)
        if (kv.second.size() > 2)
          fail(TNC_E_INVALID, "label " + std::to_string(kv.first) + " is held by more than two tensors");
      n->out_label.assign(d->out_label, d->out_label + d->n_qubits);
      std::set<int32_t> outs;
      for (auto x : n->out_label) {
        auto it = n->holders.find(x);
        if (it == n->holders.end() || it->second.size() != 1)
          fail(TNC_E_INVALID, "output label " + std::to_string(x) + " must be held by exactly one tensor");
        if (!outs.insert(x).second) fail(TNC_E_INVALID, "two qubits share an output label");
      }
      for (auto& kv : n->holders)
        if (kv.second.size() == 1 && !outs.count(kv.first))
          fail(TNC_E_INVALID, "label " + std::to_string(kv.first) + " is dangling (one holder, not an output)");
      n->slice_ids = {0, 0};
      n->closed = {0};
    } catch (...) {
      delete n;
      throw;
    }
    *out = n;
  });
}

tnc_status tnc_net_set_path(tnc_net net, const int32_t* pairs, int32_t n, const int32_t* out_orders) {
  return guard([&] {
    if (!net) fail(TNC_E_NOT_FOUND, "null network");
    if (out_orders) fail(TNC_E_UNSUPPORTED, "explicit result orders are not supported; pass NULL");
    if (n < 0 || (n > 0 && !pairs)) fail(TNC_E_INVALID, "bad path array");
    const int nt = int(net->labels.size());
    std::vector<bool> alive(nt, true);
    std::vector<std::pair<int, int>> path;
    for (int s = 0; s < n; ++s) {
      const int i = pairs[2 * s], j = pairs[2 * s + 1];
      if (i < 0 || j < 0 || i >= nt || j >= nt || i == j)
        fail(TNC_E_INVALID, "path step " + std::to_string(s) + " has an invalid pair");
      if (!alive[i] || !alive[j])
        fail(TNC_E_INVALID, "path step " + std::to_string(s) + " uses a retired tensor");
      alive[j] = false;
      path.push_back({i, j});
    }
    int left = 0;
    for (bool a : alive) left += a;
    if (left != 1) fail(TNC_E_INVALID, "the path leaves " + std::to_string(left) + " tensors (need 1)");
    net->path = path;
    net->has_path = true;
  });
}

static void set_slices(tnc_net net, const int32_t* sliced, int32_t k, const uint64_t* ids,
                       int64_t n_ids, int words) {
  if (!net) fail(TNC_E_NOT_FOUND, "null network");
  const int kmax = words == 1 ? 63 : 127;
  if (k < 0 || k > kmax) fail(TNC_E_INVALID, "k must be in [0, " + std::to_string(kmax) + "]");
  if (n_ids < 1 || !ids || (k > 0 && !sliced)) fail(TNC_E_INVALID, "bad slice arrays");
  std::set<int32_t> outs(net->out_label.begin(), net->out_label.end()), seen;
  for (int b = 0; b < k; ++b) {
    auto it = net->holders.find(sliced[b]);
    if (it == net->holders.end() || it->second.size() != 2 || outs.count(sliced[b]))
      fail(TNC_E_INVALID, "sliced label " + std::to_string(sliced[b]) + " is not a bond");
    if (!seen.insert(sliced[b]).second) fail(TNC_E_INVALID, "a label is sliced twice");
  }
  std::vector<uint64_t> v(size_t(2 * n_ids), 0);
  for (int64_t i = 0; i < n_ids; ++i) {
    const uint64_t lo = ids[i * words], hi = words == 2 ? ids[i * words + 1] : 0;
    const bool ok = k >= 64 ? (k == 128 || (hi >> (k - 64)) == 0) : (hi == 0 && (lo >> k) == 0);
    if (!ok) fail(TNC_E_INVALID, "slice id out of range");
    v[size_t(2 * i)] = lo;
    v[size_t(2 * i + 1)] = hi;
  }
  net->sliced.assign(sliced, sliced + k);
  net->slice_ids = std::move(v);
  net->has_slices = true;
}

tnc_status tnc_net_set_slices(tnc_net net, const int32_t* sliced, int32_t k, const uint64_t* ids,
                              int64_t n_ids) {
  return guard([&] { set_slices(net, sliced, k, ids, n_ids, 1); });
}

tnc_status tnc_net_set_slices_wide(tnc_net net, const int32_t* sliced, int32_t k,
                                   const uint64_t* ids, int64_t n_ids) {
  return guard([&] { set_slices(net, sliced, k, ids, n_ids, 2); });
}

tnc_status tnc_net_set_targets(tnc_net net, const int32_t* open, int32_t n_open,
                               const uint64_t* closed, int64_t L) {
  return guard([&] {
    if (!net) fail(TNC_E_NOT_FOUND, "null network");
    const int n = net->n_qubits;
    if (n_open < 0 || n_open > n || (n_open > 0 && !open)) fail(TNC_E_INVALID, "bad open-qubit list");
    if (n_open > 30) fail(TNC_E_UNSUPPORTED, "more than 30 open qubits");
    if (L < 1 || !closed) fail(TNC_E_INVALID, "need at least one group");
    std::set<int32_t> os;
    uint64_t omask = 0;
    for (int t = 0; t < n_open; ++t) {
      if (open[t] < 0 || open[t] >= n) fail(TNC_E_INVALID, "open qubit out of range");
      if (!os.insert(open[t]).second) fail(TNC_E_INVALID, "open qubit listed twice");
      omask |= uint64_t(1) << (n - 1 - open[t]);
    }
    const uint64_t nmask = n == 64 ? ~uint64_t(0) : ((uint64_t(1) << n) - 1);
    std::vector<uint64_t> c(closed, closed + L);
    for (auto& x : c) x &= nmask & ~omask;
    std::vector<uint64_t> s = c;
    std::sort(s.begin(), s.end());
    if (std::adjacent_find(s.begin(), s.end()) != s.end())
      fail(TNC_E_INVALID, "two groups have the same closed bits");
    net->open.assign(open, open + n_open);
    net->closed = c;
    net->has_targets = true;
  });
}

tnc_status tnc_plan_create(tnc_net net, tnc_precision precision, int32_t max_batch, tnc_plan* out) {
  return guard([&] {
    if (!net || !out) fail(TNC_E_INVALID, "null argument");
    *out = nullptr;
    *out = make_plan(*net, precision, max_batch);
  });
}

tnc_status tnc_plan_workspace_bytes(tnc_plan p, uint64_t* bytes) {
  return guard([&] {
    if (!p || !bytes) fail(TNC_E_INVALID, "null argument");
    *bytes = p->ws_bytes;
  });
}

tnc_status tnc_plan_stats(tnc_plan p, double* flops, double* bytes, int32_t* n_steps) {
  return guard([&] {
    if (!p) fail(TNC_E_INVALID, "null plan");
    if (flops) *flops = p->flops_slice;
    if (bytes) *bytes = p->bytes_slice;
    if (n_steps) *n_steps = p->n_steps;
  });
}

tnc_status tnc_plan_work(tnc_plan p, int64_t first, int64_t count, double* flops) {
  return guard([&] {
    if (!p || !flops) fail(TNC_E_INVALID, "null argument");
    if (first < 0 || count < 0 || first + count > p->n_slices())
      fail(TNC_E_INVALID, "slice range out of bounds");
    *flops = plan_work(*p, first, count);
  });
}

static void check_ws(tnc_plan p, void* ws, uint64_t bytes) {
  if (!ws) fail(TNC_E_INVALID, "null workspace");
  if (bytes < p->ws_bytes)
    fail(TNC_E_OOM, "workspace of " + std::to_string(bytes) + " bytes < required " + std::to_string(p->ws_bytes));
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) fail(TNC_E_INVALID, "workspace must be 256-byte aligned");
}

tnc_status tnc_contract_range(tnc_plan p, void* ws, uint64_t ws_bytes, void* stream, double* amps,
                              int64_t first, int64_t count, int32_t accumulate) {
  return guard([&] {
    if (!p || !amps) fail(TNC_E_INVALID, "null argument");
    check_ws(p, ws, ws_bytes);
    if (first < 0 || count < 0 || first + count > p->n_slices())
      fail(TNC_E_INVALID, "slice range outside the slice list");
    DeviceGuard dg(p->device);
    Exec e{*p, static_cast<uint8_t*>(ws), static_cast<hipStream_t>(stream)};
    e.contract(amps, first, count, accumulate != 0);
  });
}

tnc_status tnc_contract(tnc_plan p, void* ws, uint64_t ws_bytes, void* stream, double* amps,
                        double* h_norm) {
  return guard([&] {
    if (!p || !amps) fail(TNC_E_INVALID, "null argument");
    check_ws(p, ws, ws_bytes);
    DeviceGuard dg(p->device);
    Exec e{*p, static_cast<uint8_t*>(ws), static_cast<hipStream_t>(stream)};
    e.contract(amps, 0, p->n_slices(), false);
    if (h_norm) {
      double* parts = reinterpret_cast<double*>(e.ws + p->bufs[p->b_norm].off);
      hipError_t err = launch_norm(amps, p->L << p->n_open, parts, p->norm_parts,
                                   parts + p->norm_parts, e.s);
      if (err != hipSuccess) fail(TNC_E_HIP, hipGetErrorString(err));
      HIPCHK(hipMemcpyAsync(h_norm, parts + p->norm_parts, 8, hipMemcpyDeviceToHost, e.s));
      HIPCHK(hipStreamSynchronize(e.s));
    }
  });
}

tnc_status tnc_sample(tnc_plan p, void* ws, uint64_t ws_bytes, const double* amps, uint64_t seed,
                      int64_t n_samples, uint64_t* h_bits, void* stream) {
  return guard([&] {
    if (!p || !amps || (n_samples > 0 && !h_bits)) fail(TNC_E_INVALID, "null argument");
    check_ws(p, ws, ws_bytes);
    DeviceGuard dg(p->device);
    sample_into(*p, static_cast<uint8_t*>(ws), amps, seed, n_samples, h_bits,
                static_cast<hipStream_t>(stream));
  });
}

tnc_status tnc_sample_metropolis(tnc_plan p, void* ws, uint64_t ws_bytes, const double* amps,
                                 uint64_t seed, int64_t n_samples, int32_t steps,
                                 uint64_t* h_bits, void* stream) {
  return guard([&] {
    if (!p || !amps || (n_samples > 0 && !h_bits)) fail(TNC_E_INVALID, "null argument");
    check_ws(p, ws, ws_bytes);
    DeviceGuard dg(p->device);
    sample_chain_into(*p, static_cast<uint8_t*>(ws), amps, seed, n_samples, false, steps, 0.0,
                      h_bits, static_cast<hipStream_t>(stream));
  });
}

tnc_status tnc_sample_frugal(tnc_plan p, void* ws, uint64_t ws_bytes, const double* amps,
                             uint64_t seed, int64_t n_samples, double m, int32_t max_trials,
                             uint64_t* h_bits, void* stream) {
  return guard([&] {
    if (!p || !amps || (n_samples > 0 && !h_bits)) fail(TNC_E_INVALID, "null argument");
    check_ws(p, ws, ws_bytes);
    DeviceGuard dg(p->device);
    sample_chain_into(*p, static_cast<uint8_t*>(ws), amps, seed, n_samples, true, max_trials, m,
                      h_bits, static_cast<hipStream_t>(stream));
  });
}

tnc_status tnc_plan_destroy(tnc_plan p) {
  return guard([&] { delete p; });
}

tnc_status tnc_net_destroy(tnc_net n) {
  return guard([&] { delete n; });
}

tnc_status tnc_plan_n_launches(tnc_plan p, int32_t* n) {
  return guard([&] {
    if (!p || !n) fail(TNC_E_INVALID, "null argument");
    *n = int32_t(p->inv.size() + p->dep.size());
  });
}

tnc_status tnc_plan_launch_info(tnc_plan p, int32_t i, tnc_step_info* info) {
  return guard([&] {
    if (!p || !info) fail(TNC_E_INVALID, "null argument");
    const int P = int(p->inv.size());
    if (i < 0 || i >= P + int(p->dep.size())) fail(TNC_E_INVALID, "launch index out of range");
    const Launch& L = i < P ? p->inv[i] : p->dep[i - P];
    *info = L.info;
    info->kind = L.kind;
    info->invariant = L.inv ? 1 : (L.shared ? 2 : 0);
    info->config = info->k_splits = info->row_mode = info->reserved = 0;
    if (L.kind == K_GEMM) {
      info->config = L.gm.config;
      info->k_splits = L.gm.k_splits;
      info->row_mode = L.stk_off >= 0 ? 2 : (L.gm.fold ? 1 : 0);
    }
  });
}

tnc_status tnc_plan_batch_slices(tnc_plan p, int32_t* batch) {
  return guard([&] {
    if (!p || !batch) fail(TNC_E_INVALID, "null argument");
    *batch = p->batch;
  });
}

tnc_status tnc_plan_autotune(tnc_plan p, void* ws, uint64_t ws_bytes, void* stream, int32_t reps,
                             int32_t* n_changed) {
  return guard([&] {
    if (!p) fail(TNC_E_INVALID, "null plan");
    check_ws(p, ws, ws_bytes);
    if (reps < 1) fail(TNC_E_INVALID, "reps must be >= 1");
    DeviceGuard dg(p->device);
    const int c = autotune(*p, static_cast<uint8_t*>(ws), static_cast<hipStream_t>(stream), reps);
    if (n_changed) *n_changed = c;
  });
}

tnc_status tnc_plan_set_timing(tnc_plan p, int32_t enable) {
  return guard([&] {
    if (!p) fail(TNC_E_INVALID, "null plan");
    p->timing = enable != 0;
  });
}

tnc_status tnc_plan_timing(tnc_plan p, double* ms, double* bytes, double* flops, int64_t* launches,
                           int32_t reset) {
  return guard([&] {
    if (!p) fail(TNC_E_INVALID, "null plan");
    DeviceGuard dg(p->device);
    harvest(*p);
    for (int k = 0; k < kKinds; ++k) {
      if (ms) ms[k] = p->t_ms[k];
      if (bytes) bytes[k] = p->t_bytes[k];
      if (flops) flops[k] = p->t_flops[k];
      if (launches) launches[k] = p->t_n[k];
    }
    if (reset) {
      for (int k = 0; k < kKinds; ++k) p->t_ms[k] = p->t_bytes[k] = p->t_flops[k] = 0, p->t_n[k] = 0;
      std::fill(p->l_ms.begin(), p->l_ms.end(), 0.0);
      std::fill(p->l_n.begin(), p->l_n.end(), 0);
    }
  });
}

tnc_status tnc_plan_launch_timing(tnc_plan p, int32_t i, double* ms, int64_t* launches) {
  return guard([&] {
    if (!p) fail(TNC_E_INVALID, "null plan");
    const int n = int(p->inv.size() + p->dep.size());
    if (i < 0 || i >= n) fail(TNC_E_INVALID, "launch index out of range");
    DeviceGuard dg(p->device);
    harvest(*p);
    const bool have = p->l_ms.size() == size_t(n);
    if (ms) *ms = have ? p->l_ms[size_t(i)] : 0.0;
    if (launches) *launches = have ? p->l_n[size_t(i)] : 0;
  });
}


tnc_status tnc_server_create(int device, void* d_arena, uint64_t arena_bytes, int32_t max_slots,
                             int32_t chunk_batches, tnc_server* out) {
  return guard([&] {
    if (!out || !d_arena) fail(TNC_E_INVALID, "null argument");
    *out = nullptr;
    if (max_slots < 1 || max_slots > 64) fail(TNC_E_INVALID, "max_slots must be in [1, 64]");
    if (chunk_batches < 1) fail(TNC_E_INVALID, "chunk_batches must be >= 1");
    if (reinterpret_cast<uintptr_t>(d_arena) % kAlign) fail(TNC_E_INVALID, "arena must be 256-byte aligned");
    DeviceGuard dg(device);
    auto* s = new tnc_server_s();
    try {
      s->device = device;
      s->arena = static_cast<uint8_t*>(d_arena);
      s->arena_bytes = arena_bytes / kAlign * kAlign;
      s->max_slots = max_slots;
      s->chunk_batches = chunk_batches;
      s->free_list[0] = s->arena_bytes;
      s->slot_busy.assign(size_t(max_slots), false);
      s->pin.assign(size_t(max_slots), nullptr);
      s->pin_cap.assign(size_t(max_slots), 0);
      // TNC_FAULT=launch:N: the N-th launch unit this server enqueues (counted over all its
      // requests) fails before it is enqueued; for tests of failure isolation
      if (const char* f = std::getenv("TNC_FAULT")) {
        long long n = 0;
        if (std::sscanf(f, "launch:%lld", &n) != 1 || n < 1)
          fail(TNC_E_INVALID, "TNC_FAULT must read launch:N with N >= 1");
        s->fault_left = n;
      }
      for (int k = 0; k < max_slots; ++k) {
        hipStream_t st;
        HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        s->streams.push_back(st);
      }
      s->worker = std::thread([s] { s->run(); });
    } catch (...) {
      delete s;
      throw;
    }
    *out = s;
  });
}

tnc_status tnc_server_submit(tnc_server s, tnc_net net, tnc_precision precision,
                             int32_t max_batch_slices, int64_t n_samples, uint64_t seed,
                             uint64_t* request_id) {
  return guard([&] {
    if (!s || !net || !request_id) fail(TNC_E_INVALID, "null argument");
    auto* r = new Request();
    try {
      r->plan = make_plan(*net, precision, max_batch_slices, s->arena_bytes / uint64_t(s->max_slots));
      if (n_samples < 0) fail(TNC_E_INVALID, "negative sample count");
      if (r->plan->L > 1 && n_samples != 0 && n_samples != r->plan->L)
        fail(TNC_E_INVALID, "with several groups, n_samples must be 0 or the number of groups");
      r->n_samples = n_samples;
      r->seed = seed;
      r->ws_bytes = r->plan->ws_bytes;
      r->amps_bytes = uint64_t(r->plan->L << r->plan->n_open) * 16;
      r->footprint = align_up(r->ws_bytes) + align_up(r->amps_bytes);
      r->total = r->plan->n_slices();
      if (r->footprint > s->arena_bytes)
        fail(TNC_E_OOM, "request needs " + std::to_string(r->footprint) + " bytes, arena has " +
                            std::to_string(s->arena_bytes));
    } catch (...) {
      delete r;
      throw;
    }
    {
      std::lock_guard<std::mutex> g(s->mu);
      r->id = s->next_id++;
      r->t_submit = s->now();
      s->all[r->id] = r;
      s->pending.push_back(r);
    }
    s->cv.notify_all();
    *request_id = r->id;
  });
}

tnc_status tnc_server_poll(tnc_server s, uint64_t id, double* h_amps, uint64_t* h_bits,
                           tnc_request_info* info) {
  Request* done = nullptr;
  tnc_status st = guard([&] {
    if (!s) fail(TNC_E_INVALID, "null server");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->all.find(id);
    if (it == s->all.end()) fail(TNC_E_NOT_FOUND, "unknown request id");
    Request* r = it->second;
    // t_done is written under the lock when the worker retires the request; everything
    // the worker wrote before that is visible from here on
    const bool finished = r->t_done != 0;
    if (info) {
      info->t_submit = r->t_submit;
      info->t_admit = r->t_admit;
      info->t_done = r->t_done;
      info->n_amplitudes = r->plan->L << r->plan->n_open;
      info->n_samples = r->n_samples;
      info->norm = finished ? r->norm : 0.0;
      info->slices = r->total;
      info->footprint_bytes = double(r->footprint);
    }
    if (!finished) fail(TNC_E_BUSY, "request not finished");
    s->all.erase(it);
    done = r;
  });
  if (st != TNC_OK) return st;
  if (done->state == R_FAILED) {
    g_err = done->err;
    const tnc_status code = done->code;
    delete done;
    return code;
  }
  if (h_amps) std::memcpy(h_amps, done->amps.data(), done->amps.size() * sizeof(double));
  if (h_bits && !done->bits.empty()) std::memcpy(h_bits, done->bits.data(), done->bits.size() * 8);
  delete done;
  return TNC_OK;
}

tnc_status tnc_server_pending(tnc_server s, int32_t* queued, int32_t* running) {
  return guard([&] {
    if (!s) fail(TNC_E_INVALID, "null server");
    std::lock_guard<std::mutex> g(s->mu);
    if (queued) *queued = int32_t(s->pending.size());
    if (running) *running = int32_t(s->active.size());
  });
}

tnc_status tnc_server_destroy(tnc_server s) {
  return guard([&] { delete s; });
}

}  // extern "C"

