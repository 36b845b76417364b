/* tnc.h - C ABI of the sliced sparse-state tensor-network contractor for MI355X (gfx950).
 *
 * The library contracts the tensor network of a random quantum circuit once per slice
 * and sums the slices, in FP64, into a sparse set of output amplitudes psi_hat(s), then
 * draws bitstrings by |psi_hat(s)|^2 - the sampling method of Pan, Chen & Zhang,
 * "Solving the sampling problem of the Sycamore quantum circuits" (arXiv:2111.03011).
 *
 * Conventions shared by every call
 *   - Every call returns tnc_status; no exception or abort crosses the ABI.  On an error
 *     tnc_last_error() describes it (thread-local, valid until the next tnc_* call on the
 *     same thread).
 *   - Host arrays passed in are copied during the call; the caller keeps ownership.
 *   - Device memory is never allocated by the library for results or intermediates: the
 *     caller passes a workspace of tnc_plan_workspace_bytes() bytes and the output
 *     buffer (device pointers, e.g. from torch tensors).  Streams are hipStream_t passed
 *     as void* (NULL = the default stream).
 *   - Bit order: in a uint64 bitstring, bit (n-1-q) holds qubit q's value s_q, so qubit 0
 *     is the most significant of the n bits.  The open configuration of a group is
 *     mu = sum_t s_{open[t]} 2^(n_open-1-t): the first listed open qubit is the most
 *     significant bit of mu.
 *   - Complex numbers are interleaved (re, im).
 */
#ifndef TNC_H
#define TNC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tnc_status;
enum {
  TNC_OK = 0,
  TNC_E_INVALID = -1,      /* bad argument, network, path, slices or targets */
  TNC_E_OOM = -2,          /* workspace or arena too small */
  TNC_E_HIP = -3,          /* a HIP runtime call failed */
  TNC_E_UNSUPPORTED = -4,  /* valid request the library does not implement */
  TNC_E_BUSY = -5,         /* result not ready yet */
  TNC_E_NOT_FOUND = -6,    /* unknown handle or id */
  TNC_E_INTERNAL = -7
};

const char* tnc_last_error(void);

/* Arithmetic of the contraction steps.  The slice sum and the sampler are FP64 in every
 * case, and tensors are stored as complex64 in every case, each with a power-of-two
 * exponent per slice: the stored values times 2^E are the tensor (E and the tensor's
 * largest component are recorded by the kernel that produces it).  Operands are rescaled
 * exactly by powers of two as they are loaded, so no stored value leaves the range of the
 * arithmetic, however small a slice's amplitudes (a slice of a heavily sliced 53-qubit
 * network has amplitudes near 1e-39, below FP32's normal range); the FP64 slice sum
 * applies 2^E.
 *   TNC_C64     GEMM steps on the FP32 matrix cores, FP32 accumulation; operands whose
 *               largest component lies outside [2^-20, 2^21) are brought to [1, 2).
 *   TNC_BF16X3  GEMM steps split every operand value x into hi = bf16(x) and
 *               lo = bf16(x - hi) and accumulate hi*hi + hi*lo + lo*hi in FP32 on the BF16
 *               matrix cores (about 16 significant bits per operand; BF16 has FP32's
 *               exponent range and the same rescaling as TNC_C64).
 *   TNC_FP16X3  the same three products in FP16: every operand with largest component in
 *               [2^e, 2^(e+1)) is scaled by 2^(13 - e) before the split (|hi| < 2^14, far
 *               below FP16's limit; about 22 significant bits per operand).
 *   the 3M forms are declared for ABI stability and return TNC_E_UNSUPPORTED. */
typedef enum {
  TNC_C64 = 0,
  TNC_FP16X3 = 1,
  TNC_BF16X3 = 2,
  TNC_FP16X3_3M = 3,
  TNC_BF16X3_3M = 4
} tnc_precision;

typedef struct tnc_net_s* tnc_net;    /* opaque; freed by tnc_net_destroy */
typedef struct tnc_plan_s* tnc_plan;  /* opaque; freed by tnc_plan_destroy */

/* The tensor network of a circuit (paper, "Method": gates are matrices and four-way
 * tensors, the initial state a set of vectors, the final state a boundary).  Every bond
 * has dimension 2.  All pointers are host memory.
 *   ranks[n_tensors]      rank of each tensor (0..40)
 *   labels[sum(ranks)]    label ids (>= 0) of each tensor, concatenated; a label is held
 *                         by exactly two tensors (a bond) or by one tensor (an output leg)
 *   data                  complex128 entries of each tensor, concatenated, 2^rank each,
 *                         row-major in label order (first label slowest)
 *   out_label[n_qubits]   output-leg label of each qubit; every label held by one tensor
 *                         must be an output leg */
typedef struct {
  int32_t n_qubits;
  int32_t n_tensors;
  const int32_t* ranks;
  const int32_t* labels;
  const double* data;
  const int32_t* out_label;
} tnc_network_desc;

/* Copy a network (validated) for use on HIP device `device`. */
tnc_status tnc_net_create(int device, const tnc_network_desc* desc, tnc_net* out);

/* Contraction order (Appendix E format): n pairs (i, j); the contraction of tensors i and
 * j is stored at position i and j is retired.  After the last pair exactly one tensor must
 * remain.  out_orders must be NULL (the library chooses every result's label order). */
tnc_status tnc_net_set_path(tnc_net net, const int32_t* pairs, int32_t n,
                            const int32_t* out_orders);

/* Slicing (Appendix B.2): fix the k labels sliced_labels[0..k) and sum over the slice
 * ids.  Bit b of a slice id is the value of sliced_labels[b].  Each sliced label must be
 * a bond.  k = 0 with n_ids = 1 (id 0) means unsliced.  Ids must be < 2^k. */
tnc_status tnc_net_set_slices(tnc_net net, const int32_t* sliced_labels, int32_t k,
                              const uint64_t* slice_ids, int64_t n_ids);

/* The same with up to 127 sliced labels: slice id i is the two words
 * slice_ids[2i] (bits 0-63) and slice_ids[2i+1] (bits 64-127). */
tnc_status tnc_net_set_slices_wide(tnc_net net, const int32_t* sliced_labels, int32_t k,
                                   const uint64_t* slice_ids, int64_t n_ids);

/* Sparse-state targets (Appendix A): L groups; group i is closed_bits[i] on the closed
 * qubits joined with all 2^n_open configurations of the open qubits.  Bits of open
 * qubits in closed_bits are ignored.  Closed parts must be distinct.  n_qubits <= 64. */
tnc_status tnc_net_set_targets(tnc_net net, const int32_t* open_qubits, int32_t n_open,
                               const uint64_t* closed_bits, int64_t L);

/* Compile the step program of a network whose path, slices and targets are set.
 * max_batch_slices >= 1: slices contracted together per launch sequence (capped at the
 * slice count).  0 = automatic: the smallest power of two whose batch carries >= 2.5e11
 * flops of per-slice work, at most 256, with at most 16 GiB of workspace. */
tnc_status tnc_plan_create(tnc_net net, tnc_precision precision, int32_t max_batch_slices,
                           tnc_plan* out);

/* Slices per launch sequence the plan was compiled for. */
tnc_status tnc_plan_batch_slices(tnc_plan plan, int32_t* batch);

/* Bytes of device workspace tnc_contract needs. */
tnc_status tnc_plan_workspace_bytes(tnc_plan plan, uint64_t* bytes);

/* Algorithmic cost of one slice contracted alone: flops = 8 x complex multiply-adds
 * (Table I caption), bytes = operands read + results written by every step.  Steps that
 * touch no sliced tensor are run once per tnc_contract call and are not included. */
tnc_status tnc_plan_stats(tnc_plan plan, double* flops_per_slice, double* bytes_per_slice,
                          int32_t* n_steps);

/* Head reuse inside a batch (the paper's reuse of the head across the slices of one
 * subtask, Method and Appendix B.2): the slices of a launch sequence are consecutive in
 * the slice list, and a step whose sliced labels all keep one value across them (their
 * slice-id bits agree) is computed once per batch instead of once per slice.  Batches are
 * runs of at most max_batch_slices consecutive ids, cut short where such a bit would
 * change; with ids in counting order and the labels that vary fastest on the low bits,
 * every step above only high-bit labels is shared.  (TNC_NO_SHARE=1 in the environment at
 * plan creation turns this off.)
 * tnc_plan_work: algorithmic flops that contracting slices [first, first + count) executes,
 * shared steps counted once per batch and slice-invariant steps once. */
tnc_status tnc_plan_work(tnc_plan plan, int64_t first, int64_t count, double* flops);

/* Contract all slice ids and write the FP64 sum to d_amps (device, [L][2^n_open]
 * complex128, caller-owned).  h_norm (host, nullable) receives sum |amp|^2 (paper,
 * Results: the norm of the sparse state); it synchronises the stream. */
tnc_status tnc_contract(tnc_plan plan, void* d_workspace, uint64_t ws_bytes, void* hip_stream,
                        double* d_amps, double* h_norm);

/* Contract slice ids [first, first + count) of the slice list.  accumulate = 0 overwrites
 * d_amps with their sum, 1 adds their sum to it (summation order: ascending position). */
tnc_status tnc_contract_range(tnc_plan plan, void* d_workspace, uint64_t ws_bytes,
                              void* hip_stream, double* d_amps, int64_t first, int64_t count,
                              int32_t accumulate);

/* Draw bitstrings by |amp|^2 (main text, sampling paragraph).  d_amps: device
 * [L][2^n_open] complex128.  L == 1: n_samples draws from the one group; L > 1: n_samples
 * must equal L, one draw per group.  Uniforms: u_j = (SplitMix64 output j+1 from state
 * `seed`) >> 11 times 2^-53, j = draw index (L == 1) or group index (L > 1); the draw is the
 * smallest mu with c_mu > u * c_{l-1}, c the FP64 running sum of re^2 + im^2 in mu order.
 * h_bitstrings (host, [n_samples]) receives full bitstrings.  The workspace is the one
 * tnc_contract uses (its scratch holds the running sums).  Synchronises the stream. */
tnc_status tnc_sample(tnc_plan plan, void* d_workspace, uint64_t ws_bytes, const double* d_amps,
                      uint64_t seed, int64_t n_samples, uint64_t* h_bitstrings, void* hip_stream);

/* The paper's in-group samplers (main text, sampling paragraph), with the same draw
 * convention as tnc_sample (L == 1: n_samples independent draws from the one group;
 * L > 1: n_samples == L, draw d from group d), w_mu = re^2 + im^2 rounded as in
 * tnc_sample, u_k = (SplitMix64 output k+1 from state `seed`) >> 11 times 2^-53 and
 * floor(u l) for a uniform index.  Synchronous on the stream; the workspace is the one
 * tnc_contract uses.
 * tnc_sample_metropolis: draw d runs a Metropolis chain over its group: with
 * k0 = d (2 steps + 1) it starts at floor(u_k0 l), and step t = 1..steps proposes
 * nu = floor(u_(k0+2t-1) l) and moves iff w_nu >= u_(k0+2t) w_mu; the draw is the last
 * state.  steps >= 0.
 * tnc_sample_frugal: frugal rejection sampling: with k0 = 2 d max_trials, proposal t is
 * nu = floor(u_(k0+2t) l), accepted iff u_(k0+2t+1) (m S) < w_nu l (S = sum of w over the
 * group in mu order), i.e. with probability min(1, w_nu / (m mean w)); after max_trials
 * rejections the last proposal is the draw.  m > 0 finite, max_trials >= 1. */
tnc_status tnc_sample_metropolis(tnc_plan plan, void* d_workspace, uint64_t ws_bytes,
                                 const double* d_amps, uint64_t seed, int64_t n_samples,
                                 int32_t steps, uint64_t* h_bitstrings, void* hip_stream);
tnc_status tnc_sample_frugal(tnc_plan plan, void* d_workspace, uint64_t ws_bytes,
                             const double* d_amps, uint64_t seed, int64_t n_samples, double m,
                             int32_t max_trials, uint64_t* h_bitstrings, void* hip_stream);

/* tnc_sample for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation), and that would otherwise have
 * to keep a plan's workspace only to sample.  Same arguments, draws and uniforms as
 * tnc_sample, minus the workspace: the closed bits, open qubit ids, running sums and draws
 * live in a static device buffer of 16 MiB inside the library (one per GPU, held until the
 * process ends; nothing is allocated or freed).  A plan whose draws need more (L groups:
 * 16 bytes per group; one group: 8 bytes per amplitude plus 8 per draw in flight) is
 * rejected with TNC_E_INVALID.  Every call on one GPU shares that buffer and overwrites it:
 * calls that overlap on one GPU (from several host threads or streams) race.  Synchronous
 * on the stream. */
tnc_status tnc_sample_noalloc(tnc_plan plan, const double* d_amps, uint64_t seed,
                              int64_t n_samples, uint64_t* h_bitstrings, void* hip_stream);

tnc_status tnc_plan_destroy(tnc_plan plan);
tnc_status tnc_net_destroy(tnc_net net);

/* Per-step description for reporting: kind 1 = GEMM, 2 = small-operand stream, 3 = slice
 * leaves, 4 = slice sum, 5 = split-K reduction, 6 = clearing of the scale records (once per
 * call for slice-invariant tensors, once per batch for the others) (0 is reserved: operands
 * are never permuted, the GEMM reads them in their stored layouts); rows, m, n, k in
 * elements; flops and bytes algorithmic (one slice); invariant = 1 if run once per call,
 * 2 if run once per batch (head reuse, see tnc_plan_work), 0 if run per slice.  For GEMMs:
 * tile configuration (0 = 128x64, 1 = 128x16, 2 = 64x32, 3 = 128x128 complex), split-K
 * factor, and row mode (0 = one launch row per output row, 1 = rows folded into M because
 * the N-side operand is shared, 2 = output rows sharing an N-side row stacked along M). */
typedef struct {
  int32_t kind;
  int32_t invariant;
  int64_t rows, m, n, k;
  double flops;
  double bytes;
  int32_t config, k_splits, row_mode, reserved;
} tnc_step_info;

/* Autotuner: for every GEMM launch, time each tile configuration (and split-K factors up
 * to the one the plan sized its partial buffer for) `reps` times on this workspace and
 * stream, keep the fastest, and drop the captured graph so the next call recaptures it.
 * Results are cached per shape for the process; with TNC_TUNE_CACHE naming a file they are
 * appended there and reused by later processes.  Overwrites the workspace's intermediates
 * (contract afterwards).  n_changed (nullable) receives how many launches changed. */
tnc_status tnc_plan_autotune(tnc_plan plan, void* d_workspace, uint64_t ws_bytes, void* hip_stream,
                             int32_t reps, int32_t* n_changed);

tnc_status tnc_plan_n_launches(tnc_plan plan, int32_t* n);
tnc_status tnc_plan_launch_info(tnc_plan plan, int32_t i, tnc_step_info* info);

/* Timing of launches by kind on the contraction stream.  enable = 1 makes later
 * tnc_contract calls record a HIP event pair around every launch of a bounded sample of
 * slice batches (about 4096 launches per call; the other batches replay the graph);
 * tnc_plan_timing then returns, per kind (arrays of 7), the summed milliseconds, summed
 * algorithmic bytes and flops and the launch count since the last reset (synchronises on
 * the events). */
tnc_status tnc_plan_set_timing(tnc_plan plan, int32_t enable);
tnc_status tnc_plan_timing(tnc_plan plan, double* ms, double* bytes, double* flops,
                           int64_t* launches, int32_t reset);
/* The same per launch index i (as tnc_plan_launch_info): summed milliseconds and the
 * number of timed executions since the last reset of tnc_plan_timing. */
tnc_status tnc_plan_launch_timing(tnc_plan plan, int32_t i, double* ms, int64_t* launches);

/* Serving: a request loop on one device with continuous batching.  The caller hands over
 * one device arena; every submitted request (a network with path, slices and targets set)
 * is compiled at submission, queued, and admitted first come first served as soon as one of
 * max_slots slots and a contiguous block of the arena large enough for its footprint
 * (workspace + amplitude buffer) are free.  Admitted requests each own a HIP stream; the
 * server enqueues their slices chunk by chunk (chunk_batches slice batches at a time,
 * alternating between requests), so requests that arrive while others are on the GPU start
 * as soon as room frees up and their kernels overlap on the device.  The amplitudes of a
 * request are the same whether it runs alone or among others (same program, same order of
 * the FP64 sum).  The end of a request (its draws and the copies of amplitudes and draws to
 * pinned host staging) is enqueued and polled like its chunks, so the server's thread never
 * waits on one request while others could be fed.  For a given server, calls may come from
 * any host thread.  A request that fails (a HIP error, an invalid argument found late)
 * fails alone: its stream is drained, its arena block freed, and poll returns its status.
 * Fault injection for tests: with TNC_FAULT=launch:N in the environment when the server is
 * created, the N-th launch unit it enqueues (one batch of slice steps, eager or a graph
 * replay, or the slice-invariant phase; counted over all requests) fails with TNC_E_HIP
 * before anything of it is enqueued.  tnc_server_destroy waits for device work already
 * enqueued, then drops queued requests. */
typedef struct tnc_server_s* tnc_server;

typedef struct {
  double t_submit, t_admit, t_done;   /* seconds since tnc_server_create (t_done 0 = running) */
  int64_t n_amplitudes, n_samples, slices;
  double norm;                         /* sum |amp|^2 of the request's sparse state */
  double footprint_bytes;
} tnc_request_info;

/* d_arena: caller-owned device memory (256-byte aligned) the server sub-allocates. */
tnc_status tnc_server_create(int device, void* d_arena, uint64_t arena_bytes, int32_t max_slots,
                             int32_t chunk_batches, tnc_server* out);
/* max_batch_slices as in tnc_plan_create; with 0 the automatic batch is bounded by
 * arena_bytes / max_slots of workspace.
 * n_samples: 0 = amplitudes only; one group: any count; several groups: their number.
 * The network can be destroyed after the call.  TNC_E_OOM if the footprint exceeds the
 * whole arena (the request could never be admitted). */
tnc_status tnc_server_submit(tnc_server server, tnc_net net, tnc_precision precision,
                             int32_t max_batch_slices, int64_t n_samples, uint64_t seed,
                             uint64_t* request_id);
/* TNC_E_BUSY while queued or running (info is filled either way).  When finished the
 * request is retired: h_amps (host, [L][2^n_open] complex128, nullable) and h_bits (host,
 * [n_samples], nullable) receive the results, and its own status is returned. */
tnc_status tnc_server_poll(tnc_server server, uint64_t request_id, double* h_amps,
                           uint64_t* h_bits, tnc_request_info* info);
tnc_status tnc_server_pending(tnc_server server, int32_t* queued, int32_t* running);
tnc_status tnc_server_destroy(tnc_server server);

#ifdef __cplusplus
}
#endif

#endif /* TNC_H */
