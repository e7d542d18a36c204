/*
 * ldpc.h -- C ABI of the MI355X (gfx950) sum-product decoder for arbitrary
 * irregular LDPC codes.
 *
 * Method: J. Broulim, A. Ayriyan, V. Georgiev, H. Grigorian, "OpenCL/CUDA
 * algorithms for parallel decoding of any irregular LDPC code using GPU".
 * The decoder runs the paper's soft-decision sum-product algorithm
 * (Algorithm 2, with the message rules of Algorithm 1, the estimate of
 * Algorithms 4/6 and the syndrome of Algorithm 7) on the Tanner graph of a
 * binary parity-check matrix H (Sec. II-A, Eqs. (1)-(2)), with no bound on
 * node degree.
 *
 * Conventions shared by every entry point:
 *  - Every function returns an ldpc_status; on failure ldpc_last_error()
 *    gives a human-readable detail for the calling thread.
 *  - No C++ exception crosses this interface.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *    memory on the device that was current when the graph was created.
 *  - LLRs are L = ln(P(c=0)/P(c=1)); BPSK maps bit 0 to +1, so for an AWGN
 *    channel L = 2y/sigma^2 (the log-ratio of Algorithm 3's probabilities).
 */
#ifndef LDPC_H
#define LDPC_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define LDPC_API __attribute__((visibility("default")))
#else
#define LDPC_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque graph handle.  Immutable after creation; may be used by several
 * streams at once as long as each call has its own workspace. */
typedef struct ldpc_graph ldpc_graph;

typedef enum {
    LDPC_OK = 0,
    LDPC_E_INVAL = 1,        /* bad argument (sizes, null pointer, flags, workspace too small) */
    LDPC_E_RANGE = 2,        /* an H index is outside [0,m) x [0,n) */
    LDPC_E_DUP_EDGE = 3,     /* H lists the same (row, col) twice; H is binary (Sec. II-A) */
    LDPC_E_NOMEM = 4,        /* host or device allocation failed */
    LDPC_E_DEVICE = 5,       /* a HIP call or kernel launch failed */
    LDPC_E_UNSUPPORTED = 6   /* the request is valid but not supported by this build */
} ldpc_status;

/* Decode flags. */
enum {
    LDPC_NO_EARLY_STOP = 1u << 0, /* run exactly max_iter iterations (no syndrome stop) */
    LDPC_MSG_FP16 = 1u << 1,      /* store check->bit messages as IEEE fp16 (math stays fp32) */
    LDPC_MSG_BF16 = 1u << 2,      /* store check->bit messages as bfloat16 (math stays fp32) */
    LDPC_MSG_Q8 = 1u << 6,        /* store them as 8-bit fixed point: steps of 1/2, saturating at +-63.5
                                     (round to nearest even; math stays fp32) */
    /* Tile shape (at most one; default: chosen from the frame count).  Each
     * wavefront lane holds 1, 2 or 4 consecutive frame slots, so one memory
     * access of a wavefront spans 64, 128 or 256 frames of one edge or bit.
     * Results do not depend on the choice. */
    LDPC_LANE_SLOTS_1 = 1u << 3,
    LDPC_LANE_SLOTS_2 = 1u << 4,
    LDPC_LANE_SLOTS_4 = 1u << 5,
    /* Tail compaction (the ldpc_decode, ldpc_decode_noalloc and ldpc_simulate
     * entry points; ignored with LDPC_NO_EARLY_STOP and below 256 frame
     * slots).  After iteration 8 and every 4 iterations after it, a kernel
     * counts the frames still running; once they fit in a smaller copy of the
     * state (half or a quarter of the slots, at half or a quarter of the
     * frame slots per lane, at least one), it moves them into the smallest
     * copy that holds them and the remaining iterations run there; the
     * posteriors are copied back at the end.  Every decision is taken on the device: the call still only
     * enqueues work, never waits, and can be captured into a graph.  Results
     * are identical.  The workspace grows by three quarters of the per-slot
     * state. */
    LDPC_COMPACT_TAIL = 1u << 7
};

/* Graph flags. */
enum {
    LDPC_GRAPH_HOST_ONLY = 1u << 0 /* build the host tables only (no device copy; cannot decode) */
};

/*
 * Build the Tanner graph of H (Sec. II-A, Eqs. (1)-(2)) and copy its index
 * tables to the current HIP device.
 *
 *  m, n        rows (checks) and columns (bits) of H; both >= 1.
 *  nnz         number of ones in H (edges), 0 <= nnz < 2^31.
 *  rows, cols  host int32 arrays [nnz]: edge k joins check rows[k] and bit
 *              cols[k].  Any order; the order is kept (stable sorts) within
 *              each node's edge list, exactly as the paper's address arrays
 *              (Tables I and II) keep it.  Read only during the call.
 *  flags       0 or LDPC_GRAPH_HOST_ONLY.
 *  out         receives the new handle (owned by the caller; free with
 *              ldpc_graph_destroy).  Untouched on failure.
 *
 * Errors: INVAL (m or n < 1, nnz out of range, null pointer), RANGE (index
 * out of range), DUP_EDGE (repeated pair), NOMEM, DEVICE.
 * Rows or columns without edges are allowed (an empty check is always
 * satisfied; an empty column keeps its channel LLR).
 */
LDPC_API ldpc_status ldpc_graph_create(int32_t m, int32_t n, int64_t nnz,
                              const int32_t *rows, const int32_t *cols,
                              uint32_t flags, ldpc_graph **out);

/*
 * Build the Tanner graph of a quasi-cyclic (lifted) code and keep its base
 * matrix for circulant indexing.  The results section benchmarks protograph
 * expansions of a base code, and the further-acceleration subsection names
 * modifications of the algorithm for certain families of LDPC codes; this is
 * that family: every entry of the mb x nb base matrix is either a zero block
 * or a Z x Z circulant, so check i*Z + t joins bit j*Z + ((t + s_ij) mod Z)
 * for every base entry (i, j) with shift s_ij.
 *
 *  mb, nb      base rows and columns; both >= 1.
 *  Z           lifting size >= 1; mb*Z and nb*Z, and the edge count
 *              (nonzero base entries times Z), must stay below 2^31.
 *  shifts      host int32 array [mb][nb] (row-major): s_ij in [0, Z), or -1
 *              for a zero block.  Read only during the call.
 *  flags, out  as for ldpc_graph_create.
 *
 * The graph is the one ldpc_graph_create builds from the lifted H with each
 * check's edges in base-column order, so every entry point accepts it and
 * ldpc_graph_arrays returns the same tables.  In addition, the check passes
 * of rows of up to 16 edges compute each edge's bit from its base entry
 * instead of reading the column index (sum-product rule).  Results are
 * identical to decoding the same H built by ldpc_graph_create.
 *
 * Errors: INVAL (sizes out of range, null pointer, unknown flags), RANGE (a
 * shift outside [-1, Z)), NOMEM, DEVICE.
 */
LDPC_API ldpc_status ldpc_graph_create_qc(int32_t mb, int32_t nb, int32_t Z, const int32_t *shifts,
                                 uint32_t flags, ldpc_graph **out);

/* Release the graph and its device tables.  NULL is accepted (no-op). */
LDPC_API ldpc_status ldpc_graph_destroy(ldpc_graph *g);

/* Sizes of the graph.  Any output pointer may be NULL.  device_bytes is the
 * device memory held by the graph's index tables. */
LDPC_API ldpc_status ldpc_graph_info(const ldpc_graph *g, int64_t *m, int64_t *n, int64_t *nnz,
                            int32_t *max_check_deg, int32_t *max_bit_deg,
                            int64_t *device_bytes);

/*
 * Copy the graph's address arrays to host memory (any pointer may be NULL).
 * These are the paper's Table II / Table I arrays in compressed form:
 *
 *  row_ptr    [m+1]  edges sorted by check (stable): check i owns positions
 *                    row_ptr[i] .. row_ptr[i+1]-1 (Table II's sbar and tbar)
 *  col_idx    [nnz]  bit of each check-sorted position (Table II's vbar)
 *  col_ptr    [n+1]  edges sorted by bit (stable): bit j owns positions
 *                    col_ptr[j] .. col_ptr[j+1]-1 (Table I's s and t)
 *  row_idx    [nnz]  check of each bit-sorted position (Table I's c)
 *  csr_to_csc [nnz]  bit-sorted position of each check-sorted position
 *                    (Table II's ebar)
 */
LDPC_API ldpc_status ldpc_graph_arrays(const ldpc_graph *g, int32_t *row_ptr, int32_t *col_idx,
                              int32_t *col_ptr, int32_t *row_idx, int32_t *csr_to_csc);

/*
 * Device workspace that ldpc_decode needs for `frames` frames with `flags`.
 * The workspace holds the per-frame message state (channel and posterior
 * LLRs per bit, one message per edge, per-frame counters) and is owned by the
 * caller.  Errors: INVAL (null g/bytes, frames < 0, conflicting flags).
 */
LDPC_API ldpc_status ldpc_decode_workspace_size(const ldpc_graph *g, int32_t frames, uint32_t flags,
                                       size_t *bytes);

/*
 * Decode `frames` frames with the sum-product algorithm (Algorithm 2).
 *
 * Each iteration t = 1..max_iter is one check-node update (Algorithm 1,
 * second half) on bit->check messages formed from the previous posterior
 * (Algorithm 1, first half), then the posterior and hard decision
 * (Algorithms 4/6: bit = 1 iff posterior LLR < 0; a tie gives 0), then the
 * syndrome test (Algorithm 7).  The pass before Algorithm 2's loop counts as
 * iteration 1; there is no syndrome test before it.  Unless
 * LDPC_NO_EARLY_STOP is set, a frame stops at the first iteration whose
 * estimate is a codeword.  Messages are clamped to +-64 (the posterior is
 * not clamped).  All arithmetic is fp32; messages are stored as fp32, fp16
 * or bf16 according to flags.
 *
 *  g            graph from ldpc_graph_create (not HOST_ONLY); its device
 *               must be the current device.
 *  llr_in       device float [frames][n], channel LLRs, finite.
 *  frames       >= 0 (0 is a no-op).
 *  max_iter     >= 1.
 *  flags        LDPC_NO_EARLY_STOP | at most one of LDPC_MSG_FP16, LDPC_MSG_BF16, LDPC_MSG_Q8 |
 *               at most one LDPC_LANE_SLOTS_* tile-shape flag | LDPC_COMPACT_TAIL.
 *  bits_out     device uint8 [frames][n]: the estimate (0/1).
 *  syndrome_ok  device uint8 [frames]: 1 iff the returned estimate is a codeword.
 *  iters        device int32 [frames]: iterations run, 1..max_iter (the
 *               iteration whose estimate is returned).
 *  llr_out      device float [frames][n] posterior LLRs, or NULL.
 *  workspace    device memory of at least ldpc_decode_workspace_size bytes,
 *               256-byte aligned; caller-owned; contents are scratch.
 *  hip_stream   hipStream_t to enqueue on (NULL = default stream).
 *
 * The call only enqueues work and returns (with every flag); outputs are
 * valid once the stream has reached this point.  Inputs must not be modified and outputs
 * must not be read before then.  Errors (returned synchronously; nothing is
 * enqueued): INVAL (bad sizes or pointers, workspace too small or unaligned,
 * graph built HOST_ONLY, wrong current device), DEVICE (launch failure).
 * Non-finite LLRs are a precondition violation: the result is unspecified
 * but the call does not fault.
 */
LDPC_API ldpc_status ldpc_decode(const ldpc_graph *g, const float *llr_in, int32_t frames,
                        int32_t max_iter, uint32_t flags,
                        uint8_t *bits_out, uint8_t *syndrome_ok, int32_t *iters,
                        float *llr_out, void *workspace, size_t workspace_bytes,
                        void *hip_stream);

/*
 * ldpc_decode plus per-pass timing, for profiling.  Arguments and results are
 * those of ldpc_decode; in addition the library records HIP events on
 * hip_stream around each pass, waits for the stream to finish (this call
 * blocks), and writes the elapsed times to caller-owned host arrays:
 *   check_ms [max_iter]  check-node pass of iteration t (index t-1)
 *   bit_ms   [max_iter]  bit-node pass of iteration t
 *   edge_ms  [2]         [0] state set-up and LLR transpose,
 *                        [1] final syndrome, per-frame results and output transpose
 * Errors: those of ldpc_decode; INVAL if a timing array is NULL; DEVICE if an
 * event cannot be created or the stream fails.
 */
LDPC_API ldpc_status ldpc_decode_profiled(const ldpc_graph *g, const float *llr_in, int32_t frames,
                                          int32_t max_iter, uint32_t flags,
                                          uint8_t *bits_out, uint8_t *syndrome_ok, int32_t *iters,
                                          float *llr_out, void *workspace, size_t workspace_bytes,
                                          void *hip_stream, float *check_ms, float *bit_ms,
                                          float *edge_ms);

/*
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): ldpc_decode without a
 * workspace argument.  The decode state lives in one file-scope device array
 * of LDPC_NOALLOC_SCRATCH_BYTES per device, which the library holds from its
 * first use on that device until the process ends; the call itself allocates
 * nothing.  Arguments, results and errors are those of ldpc_decode, except:
 *  - frames whose state (ldpc_decode_workspace_size with the same flags)
 *    exceeds LDPC_NOALLOC_SCRATCH_BYTES are refused with RANGE;
 *  - DEVICE if the array's device address cannot be looked up.
 * Every call on one device uses the same array, which keeps the last call's
 * contents; a call writes every part of it before reading it, so nothing
 * needs clearing.  Calls that overlap on one device (several streams or host
 * threads) race and give undefined results: serialize them, e.g. on one
 * stream.
 */
#define LDPC_NOALLOC_SCRATCH_BYTES (128u << 20)
LDPC_API ldpc_status ldpc_decode_noalloc(const ldpc_graph *g, const float *llr_in, int32_t frames,
                                         int32_t max_iter, uint32_t flags,
                                         uint8_t *bits_out, uint8_t *syndrome_ok, int32_t *iters,
                                         float *llr_out, void *hip_stream);

/* ------------------------------------------------------------------------
 * Check-node rules.
 *
 * The paper's decoder is sum-product (Algorithm 1, no simplification).  Its
 * Section 3.1 names Min-Sum and adaptive normalized / offset Min-Sum (Wu,
 * Song, Jiang, Zhao, IEEE Commun. Lett. 14(7), 2010) as derived decoders that
 * suit the same edge-level approach.  They keep the bit rule and the sign of
 * the check rule and replace the magnitude phi(sum phi(|Q|)) over the other
 * bits of the check by m = min |Q| over the other bits:
 *   LDPC_RULE_MIN_SUM_NORMALIZED  |R| = alpha * m, param = alpha in (0, 1]
 *                                 (alpha = 1 is plain Min-Sum);
 *   LDPC_RULE_MIN_SUM_OFFSET      |R| = max(m - beta, 0), param = beta in [0, 64).
 * |R| is clamped to 64 as for sum-product; a degree-1 check sends +64.
 * The arithmetic is fp32 (the products alpha * m and differences m - beta
 * are rounded once); storage follows the LDPC_MSG_* flags.
 * ------------------------------------------------------------------------ */
typedef enum {
    LDPC_RULE_SUM_PRODUCT = 0,
    LDPC_RULE_MIN_SUM_NORMALIZED = 1,
    LDPC_RULE_MIN_SUM_OFFSET = 2
} ldpc_rule_kind;

typedef struct {
    int32_t kind;          /* ldpc_rule_kind */
    float param;           /* alpha or beta; ignored for sum-product */
    int32_t reserved[2];   /* must be 0 */
} ldpc_rule;

/*
 * ldpc_decode with a selectable check rule.  rule (host pointer, read during
 * the call) may be NULL for sum-product; every other argument and the results
 * are those of ldpc_decode, including the workspace size.  Errors: those of
 * ldpc_decode; INVAL for an unknown kind, a parameter out of range or
 * non-zero reserved fields.
 */
LDPC_API ldpc_status ldpc_decode_rule(const ldpc_graph *g, const float *llr_in, int32_t frames,
                                      int32_t max_iter, uint32_t flags, const ldpc_rule *rule,
                                      uint8_t *bits_out, uint8_t *syndrome_ok, int32_t *iters,
                                      float *llr_out, void *workspace, size_t workspace_bytes,
                                      void *hip_stream);

/* ------------------------------------------------------------------------
 * Monte-Carlo error-rate runs on the device (the paper's error-rate
 * simulation: channel, decode and error count, Sec. IV and V-A).
 *
 * Each frame sends the all-zero codeword over BPSK/AWGN: every bit is sent as
 * +1 and receives y = 1 + sigma z, with sigma^2 = 1 / (2 R 10^(EbN0/10)) and
 * the nominal rate R = (n - m)/n (Eqs. (3)-(4)); the decoder input is
 * L = 2y / sigma^2.  The noise z comes from a counter-based generator, so a
 * frame's noise depends only on (seed, frame index) and a run may be split
 * over calls (first_frame) or repeated exactly:
 *   Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 *   easy as 1, 2, 3", SC 2011) with key = (seed & 0xffffffff, seed >> 32) and
 *   counter = (q, f & 0xffffffff, f >> 32, 0) for bits 4q..4q+3 of global
 *   frame f = first_frame + i; its outputs x0..x3 give uniforms
 *   u = ((x >> 9) + 0.5) 2^-23, and the Box-Muller transform of (u0, u1)
 *   gives z for bits 4q and 4q+1 (r cos(2 pi u1), r sin(2 pi u1) with
 *   r = sqrt(-2 ln u0)), that of (u2, u3) bits 4q+2 and 4q+3.
 * Frames are decoded exactly as by ldpc_decode with the same flags.  A
 * frame's bit errors are the bits whose estimate is 1 (Lpost < 0); it is a
 * frame error when that count is non-zero, and an undetected error when its
 * estimate nevertheless passed the syndrome (a different codeword).
 * ------------------------------------------------------------------------ */
typedef struct {
    uint64_t frames;        /* frames decoded */
    uint64_t frame_errors;  /* frames whose estimate differs from the codeword sent */
    uint64_t bit_errors;    /* code bits in error, summed over frames */
    uint64_t undetected;    /* frame errors whose estimate passed the syndrome */
    uint64_t iterations;    /* iteration counts, summed over frames */
} ldpc_sim_counts;

/* Workspace bytes ldpc_simulate needs for `frames` frames (0 for frames = 0). */
LDPC_API ldpc_status ldpc_simulate_workspace_size(const ldpc_graph *g, int32_t frames, uint32_t flags,
                                                  size_t *bytes);

/*
 * Draw `frames` frames (global indices first_frame .. first_frame+frames-1),
 * decode them and add their counts to *counts.  Asynchronous on hip_stream.
 *  counts     device pointer, added to atomically (zero it before a new run).
 *  llr_out    device [frames][n] float (the channel LLRs drawn), or NULL.
 *  workspace  device, 256-byte aligned, >= ldpc_simulate_workspace_size bytes.
 * flags: those of ldpc_decode.  Errors: INVAL (NULL graph/counts/workspace,
 * frames < 0, max_iter < 1, bad flags, n <= m, Eb/N0 not finite, small or
 * misaligned workspace, wrong device), DEVICE (launch failure).
 */
LDPC_API ldpc_status ldpc_simulate(const ldpc_graph *g, int32_t frames, double ebn0_db, uint64_t seed,
                                   uint64_t first_frame, int32_t max_iter, uint32_t flags,
                                   ldpc_sim_counts *counts, float *llr_out, void *workspace,
                                   size_t workspace_bytes, void *hip_stream);

/* ldpc_simulate with a selectable check rule (NULL: sum-product); the
 * arguments, counts and errors are those of ldpc_simulate and ldpc_decode_rule. */
LDPC_API ldpc_status ldpc_simulate_rule(const ldpc_graph *g, int32_t frames, double ebn0_db, uint64_t seed,
                                        uint64_t first_frame, int32_t max_iter, uint32_t flags,
                                        const ldpc_rule *rule, ldpc_sim_counts *counts, float *llr_out,
                                        void *workspace, size_t workspace_bytes, void *hip_stream);

/* ------------------------------------------------------------------------
 * Batched decoding with continuous refill.
 *
 * An engine decodes frames of several codes (graphs) in one launch sequence.
 * Each graph gets a pool of frame slots in HBM that keep the per-frame state
 * of ldpc_decode (channel and posterior LLRs per bit, one message per edge).
 * Frames are queued per graph; a decode *step* is, over every graph at once,
 * one or more iterations (iters_per_step) of a check pass and a bit pass (the
 * same arithmetic and order as ldpc_decode, Algorithm 2's loop body, with the
 * per-frame stop test of Algorithm 7 or max_iter in the bit pass: a frame that
 * stops sits out the step's remaining passes), then the output of frames that
 * stopped and the admission of queued frames into the freed slots.  Frames of
 * one graph therefore advance at their own pace: a frame's result is
 * bit-identical to decoding it alone with ldpc_decode (ldpc_decode_rule for a
 * Min-Sum rule) and the same flags.  Steps are captured once into a hipGraph
 * and replayed.
 *
 * Repacking: once a graph has no queued frames left, the frames still running
 * tend to be scattered over the pool, and every slot group holding one of
 * them costs a full pass over its messages.  When at most half of the slots
 * below the highest occupied one hold frames, the engine moves the frames
 * above the first A slots (A = frames running) into the free slots below A,
 * with their messages and LLRs, so later passes touch A slots only.  Moving a
 * frame between slots does not change its arithmetic.
 *
 * The engine owns its device memory (allocated at creation) and a HIP stream
 * of default priority; all of its work runs on that stream.  One engine must
 * not be driven from several host threads at once.
 * ------------------------------------------------------------------------ */
typedef struct ldpc_engine ldpc_engine;

/* One queued frame.  All pointers are device pointers on the engine's device. */
typedef struct {
    const float *llr;     /* [n] channel LLRs; read when the frame enters a slot */
    uint8_t *bits;        /* [n] estimate (written when the frame finishes) */
    uint8_t *ok;          /* 1 byte: 1 iff the estimate is a codeword */
    int32_t *iters;       /* 1 int32: iterations run (1..max_iter) */
    float *llr_out;       /* [n] posterior LLRs, or NULL */
    int32_t *done;        /* int32 counter incremented atomically when the frame finishes, or NULL */
} ldpc_frame;

typedef struct {
    int32_t lane_slots;   /* frame slots per wavefront lane: 1, 2 or 4; 0 = 4 */
    int32_t graph_steps;  /* decode steps per captured hipGraph replay; 0 = 8 */
    int32_t no_compaction;/* 1: never repack frames into the low slots (see below); 0 = repack */
    int32_t iters_per_step;/* decoder iterations per step (1..16; 0 = 1).  Stopped frames leave
                             their slot, and queued frames enter, once per step, so more
                             iterations per step spend fewer launches on that bookkeeping
                             but keep finished frames in their slots longer */
    int32_t rule;         /* check rule, an ldpc_rule_kind (0 = sum-product) */
    float rule_param;     /* its parameter (alpha or beta, as for ldpc_decode_rule) */
    int32_t reserved[2];  /* must be 0 */
} ldpc_engine_opts;

/*
 * Create an engine for `ngraphs` graphs (1..32).
 *  graphs      [ngraphs] graph handles (not HOST_ONLY), all on the current device;
 *              they must outlive the engine.
 *  slots       [ngraphs] slot-pool size per graph (>= 1; rounded up to a multiple
 *              of 64 * lane_slots).
 *  queue_cap   [ngraphs] queue capacity per graph (>= 1): frames submitted but not
 *              yet admitted to a slot.
 *  max_iter    1..2^30-1; flags: LDPC_NO_EARLY_STOP, LDPC_MSG_FP16 / LDPC_MSG_BF16 / LDPC_MSG_Q8.
 *  opts        may be NULL.
 * Errors: INVAL, NOMEM (device memory), DEVICE.
 */
LDPC_API ldpc_status ldpc_engine_create(const ldpc_graph *const *graphs, int32_t ngraphs,
                                        const int32_t *slots, const int32_t *queue_cap,
                                        int32_t max_iter, uint32_t flags,
                                        const ldpc_engine_opts *opts, ldpc_engine **out);

/* Release the engine (waits for its stream first).  NULL is a no-op. */
LDPC_API ldpc_status ldpc_engine_destroy(ldpc_engine *e);

/* Device memory held by the engine, and the rounded slot count of each graph
 * (slots may be NULL; otherwise [ngraphs]). */
LDPC_API ldpc_status ldpc_engine_info(const ldpc_engine *e, int64_t *device_bytes, int32_t *slots);

/*
 * Queue `count` frames (host array of descriptors, copied) for graph `graph`.
 * If hip_stream is not NULL, the engine waits for work already enqueued on it
 * (so LLRs produced there are ready) before admitting these frames.
 * Errors: INVAL (bad index, count < 0, more frames than free queue capacity:
 * nothing is queued then), DEVICE.
 */
LDPC_API ldpc_status ldpc_engine_submit(ldpc_engine *e, int32_t graph, const ldpc_frame *frames,
                                        int32_t count, void *hip_stream);

/* Free queue capacity of `graph`, from the newest queue counters the engine
 * has seen: those of the last ldpc_engine_poll/run, or of any replay already
 * finished on the device (checked without waiting). */
LDPC_API ldpc_status ldpc_engine_capacity(const ldpc_engine *e, int32_t graph, int32_t *free_entries);

/* Enqueue `replays` hipGraph replays (replays * graph_steps decode steps) on the
 * engine stream and return without waiting. */
LDPC_API ldpc_status ldpc_engine_step(ldpc_engine *e, int32_t replays);

/*
 * Wait for the engine stream, then report per graph the frames finished so
 * far (retired, [ngraphs], may be NULL) and the frames submitted but not yet
 * finished (pending, [ngraphs], may be NULL).
 */
LDPC_API ldpc_status ldpc_engine_poll(ldpc_engine *e, int64_t *retired, int64_t *pending);

/* The engine's HIP stream (owned by the engine; do not destroy it).  Work
 * enqueued on it after ldpc_engine_step runs after those steps. */
LDPC_API ldpc_status ldpc_engine_stream(const ldpc_engine *e, void **hip_stream);

/*
 * Step until every submitted frame has finished or `max_replays` replays have
 * run (0 = no limit); blocks.  replays_out (may be NULL) receives the number
 * of replays run.
 */
LDPC_API ldpc_status ldpc_engine_run(ldpc_engine *e, int32_t max_replays, int64_t *replays_out);

/*
 * Autotuner for ldpc_engine_create: times the decode of the given frames with
 * candidate tile shapes and slot-pool sizes and returns the fastest.
 * Candidates: lane_slots in {2, 4} x slot pools of {1/4, 1/2, 1} x the frame
 * count of each graph (at least one 64*lane_slots group) x (graph_steps,
 * iters_per_step) in {(4,1), (8,1), (2,2), (4,2), (1,4), (2,4)}.  Each
 * candidate engine decodes every frame twice; the second run is
 * timed.  The frames' outputs are overwritten by the trials.
 *
 *  frames[c] / frame_counts[c]  host descriptor arrays of graph c's frames
 *  slots_out [ngraphs], opts_out, best_ms (may be NULL): the winner.
 * Errors: those of ldpc_engine_create / submit / run.
 */
LDPC_API ldpc_status ldpc_engine_autotune(const ldpc_graph *const *graphs, int32_t ngraphs,
                                          const ldpc_frame *const *frames, const int32_t *frame_counts,
                                          int32_t max_iter, uint32_t flags, int32_t *slots_out,
                                          ldpc_engine_opts *opts_out, float *best_ms);

/* ------------------------------------------------------------------------
 * Serving: a request loop over an engine (continuous batching).
 *
 * Clients submit decode requests (frames of one of the server's graphs, host
 * LLRs).  A worker thread admits requests in arrival order as soon as the
 * device-memory budget, a completion counter and the graph's engine queue
 * allow, copies their LLRs to the device, and queues their frames; frames
 * enter free slots at the next engine step, so requests that arrive while
 * others are decoding share the device with them.  Finished requests are
 * copied back to host memory and time-stamped; latency = completion - submit.
 * Graphs and per-slot message state stay resident for the server's lifetime.
 * ------------------------------------------------------------------------ */
typedef struct ldpc_server ldpc_server;

typedef struct {
    int32_t lane_slots;    /* engine tile option (0 = default) */
    int32_t graph_steps;   /* engine steps per replay (0 = default) */
    int32_t max_requests;  /* requests in flight at once (0 = 4096) */
    int32_t rule;          /* check rule of the server's engine, an ldpc_rule_kind (0 = sum-product) */
    float rule_param;      /* its parameter (alpha or beta) */
    int32_t iters_per_step;/* decoder iterations per engine step (as for ldpc_engine_opts; 0 = 1) */
    int32_t reserved[2];   /* must be 0 */
} ldpc_server_opts;

/*
 * Create a server for `ngraphs` graphs with slot pools `slots` (as for
 * ldpc_engine_create) and decode settings max_iter / flags.
 *  hbm_budget   device bytes for request inputs and outputs (>= 1 MiB); a
 *               request needs about frames * n * 5 bytes.
 *  host_budget  pinned host bytes for transfers (>= 1 MiB).
 * Errors: INVAL, NOMEM, DEVICE.
 */
LDPC_API ldpc_status ldpc_server_create(const ldpc_graph *const *graphs, int32_t ngraphs, const int32_t *slots,
                                        int32_t max_iter, uint32_t flags, int64_t hbm_budget,
                                        int64_t host_budget, const ldpc_server_opts *opts, ldpc_server **out);

/* Queue a request of `frames` frames of graph `graph`; llr is host memory
 * [frames][n], copied before the call returns.  id receives the request id.
 * Errors: INVAL (bad graph, frames < 1, or a request larger than the budgets
 * or the graph's queue could ever hold), NOMEM. */
LDPC_API ldpc_status ldpc_server_submit(ldpc_server *s, int32_t graph, const float *llr, int32_t frames,
                                        int64_t *id);

/* Ids of requests completed since the last poll (up to max_ids), waiting up
 * to wait_ms milliseconds for at least one. */
LDPC_API ldpc_status ldpc_server_poll(ldpc_server *s, int64_t *ids, int32_t max_ids, int32_t *count,
                                      int32_t wait_ms);

/* Copy a completed request's results to host memory ([frames][n] bits,
 * [frames] ok, [frames] iters; any may be NULL) and its latency in seconds,
 * then release it.  Errors: INVAL (unknown or unfinished id). */
LDPC_API ldpc_status ldpc_server_result(ldpc_server *s, int64_t id, uint8_t *bits, uint8_t *ok,
                                        int32_t *iters, double *latency_s);

/* Counters: [0] submitted, [1] admitted, [2] completed, [3] frames completed,
 * [4] waiting for admission, [5] in flight, [6] device bytes in use,
 * [7] peak device bytes in use. */
LDPC_API ldpc_status ldpc_server_stats(ldpc_server *s, int64_t *stats);

/* Stop accepting requests, finish those already submitted, release everything. */
LDPC_API ldpc_status ldpc_server_destroy(ldpc_server *s);

/* Static string naming a status code. */
LDPC_API const char *ldpc_status_str(ldpc_status s);

/* Detail of the last failure on the calling thread ("" if none). */
LDPC_API const char *ldpc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LDPC_H */
