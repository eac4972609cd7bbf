/*
 * cvqkd_recon.h -- C ABI of the MI355X (gfx950) slice-reconciliation library.
 *
 * The library implements the decoding hot path of sliced reverse
 * reconciliation for CV-QKD (Ai & Malaney, arXiv 2108.08418): Bob quantises
 * his quadratures and cuts the labels into bit slices (Sec. III-B steps 1-2),
 * sends syndromes of each slice (Sec. II Step 5, Sec. III-B steps 2-3),
 * Alice forms slice LLRs from her quadratures and the slices she already
 * holds (Sec. III-B step 4) and belief-propagation decodes every sub-block of
 * length N_R independently (Sec. III-A, Sec. III-C).
 *
 * General rules
 *  - Every data pointer marked "device" is device memory of the current HIP
 *    device, owned by the caller; the library never allocates or frees it.
 *    Pointers marked "host" are read during the call only.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls that take a
 *    stream only enqueue work: they neither allocate nor synchronise, so they
 *    may be captured in a HIP graph.  Code and batch handles are created
 *    synchronously and own device copies of their tables.
 *  - Argument errors are detected on the host before anything is enqueued and
 *    return CVR_EINVAL; a failed launch returns CVR_EHIP.  Asynchronous device
 *    errors surface at a later call or at stream synchronisation.  The text of
 *    the last error of the calling thread is available from cvr_last_error().
 *  - An LLR is ln P(bit = 0) / P(bit = 1); bit 0 is sent as +1.  A hard
 *    decision is 1 iff the LLR is < 0 (so +0 and -0 both decide 0, and both
 *    have magnitude 0 in the check rules).  Bits travel as one uint8 (0/1)
 *    per bit.
 *  - Only bit 0 of every input bit byte is used.
 */
#ifndef CVQKD_RECON_H
#define CVQKD_RECON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CVR_OK = 0,
    CVR_EINVAL = -1,          /* invalid argument (nothing was enqueued)            */
    CVR_ENOMEM = -2,          /* device allocation or workspace too small           */
    CVR_EHIP = -3,            /* a HIP runtime call or kernel launch failed         */
    CVR_EUNSUPPORTED = -4     /* valid request the library does not implement       */
} cvr_status;

enum { CVR_GRAY = 0, CVR_BINARY = 1 };           /* labelling of quantiser intervals   */
enum { CVR_SP = 0, CVR_NMS = 1 };                /* check-node rule                    */
enum { CVR_F64 = 0, CVR_F32 = 1, CVR_F16 = 2 };  /* arithmetic / storage precisions    */

/* Text of the calling thread's last non-OK status ("" if none). */
const char* cvr_last_error(void);

/* Library ABI version (major * 10000 + minor * 100 + patch). */
int32_t cvr_version(void);

/* ------------------------------------------------------------------------- */
/* Parity-check matrices                                                      */
/* ------------------------------------------------------------------------- */
/* An LDPC matrix H_j shared by all sub-blocks of slice j (Sec. III-B, last
 * sentence of the step list; Sec. III-C defines G, the number of nonzeros).  */
typedef struct cvr_code_s* cvr_code_t;

/* Explicit H with m checks and n variables in CSR form (host arrays):
 * row c holds columns col_idx[row_ptr[c] .. row_ptr[c+1]-1], strictly
 * ascending, each in [0, n).  edge_type (host [E] or NULL = all 0) gives the
 * class of every edge, used to index per-type min-sum weights; values must be
 * < n_types (1 <= n_types <= 16).  Requires n >= 1, m >= 1, every row degree in
 * [1, 32].  The handle owns device copies; destroy it with cvr_code_destroy. */
cvr_status cvr_code_create_csr(int32_t n, int32_t m, const int32_t* row_ptr,
                               const int32_t* col_idx, const uint8_t* edge_type,
                               int32_t n_types, cvr_code_t* out);

/* Quasi-cyclic H lifted from an mb x nb protograph with Z x Z circulants
 * (host arrays, row-major [mb * nb]): shift = -1 marks a zero block, else
 * 0 <= shift < Z and check i*Z + k is connected to variable
 * j*Z + (k + shift) mod Z.  block_type (or NULL = 0) is the edge class of every
 * edge of the block.  n = nb*Z, m = mb*Z.  Same limits as the CSR form.      */
cvr_status cvr_code_create_qc(int32_t nb, int32_t mb, int32_t Z, const int32_t* shift,
                              const uint8_t* block_type, int32_t n_types, cvr_code_t* out);

/* Dimensions of a code (any output pointer may be NULL). */
cvr_status cvr_code_info(cvr_code_t code, int32_t* n, int32_t* m, int64_t* n_edges,
                         int32_t* n_types, int32_t* is_qc);

/* Frees the device copies.  Must not be called while work using it is queued. */
cvr_status cvr_code_destroy(cvr_code_t code);

/* ------------------------------------------------------------------------- */
/* Bob: quantiser and slices                                                  */
/* ------------------------------------------------------------------------- */
/* The quantiser M(.) of Sec. III-B step 1 and the slices of step 2.
 * y: device fp64 [n].  thresholds: host fp64 [2^m_bits - 1], strictly
 * ascending and finite (t_0 = -inf and t_{2^m} = +inf are implicit).
 * Interval index k = #{i : t_i <= y} (a value on a threshold goes up);
 * label = k xor (k >> 1) for CVR_GRAY (the Gray labelling of Sec. II Step 4)
 * or k for CVR_BINARY; slices: device uint8 [m_bits][n], row j = bit j of the
 * label (j = 0 is the least significant bit l_0).  NaN y is an input error
 * whose slices are unspecified.  1 <= m_bits <= 8; n = 0 is a no-op.        */
cvr_status slice_quantize(const double* y, int64_t n, const double* thresholds,
                          int32_t m_bits, int32_t labelling, uint8_t* slices, void* stream);

/* ------------------------------------------------------------------------- */
/* Alice: slice log-likelihood ratios                                         */
/* ------------------------------------------------------------------------- */
/* Sec. III-B step 4: Alice's soft information on Bob's slice j from her
 * quadrature x (Y = x + N(0, sigma_n^2), Sec. V) and the slices she already
 * holds (the rows of `slices` selected by known_mask):
 *   L_j = ln sum_{k in K0} P_k(x) - ln sum_{k in K1} P_k(x),
 *   P_k(x) = Pr(t_k <= Y < t_{k+1} | x),
 * K_b = intervals whose label has bit j = b and agrees with every known bit of
 * the sample.  Computed in fp64 in the log domain (tail probabilities via
 * erfc / scaled erfc) so that far tails stay finite.
 * x: device fp64 [n]; slices: device uint8 [m_bits][n] (only rows in
 * known_mask are read; may be NULL when known_mask == 0); llr_out: device
 * [n] of out_dtype (CVR_F32 or CVR_F64).  Requires sigma_n > 0, 0 <= j < m_bits,
 * bit j of known_mask clear, known_mask < 2^m_bits.                         */
cvr_status slice_llr(const double* x, int64_t n, double sigma_n, const double* thresholds,
                     int32_t m_bits, int32_t labelling, int32_t j, uint32_t known_mask,
                     const uint8_t* slices, int32_t out_dtype, void* llr_out, void* stream);

/* Sec. III-B step 4 read literally: the soft decoding output (the final LLR)
 * of lower slices enters the LLR of slice j as an a-priori weight.  As
 * slice_llr, with every interval k of K_b also weighted by
 *   prod_{i in prior_mask} Pr(S_i = bit i of label k),
 *   Pr(S_i = 0) = 1 / (1 + e^-lambda_i),  Pr(S_i = 1) = 1 / (1 + e^lambda_i),
 * lambda_i = prior_llr[i][sample] (an LLR ln P(0)/P(1), e.g. the decoder's
 * posterior of slice i).  Slices in known_mask are hard constraints as in
 * slice_llr.  A prior of +-inf is a hard bit (the same result as holding the
 * slice in known_mask); lambda = 0 for every prior slice gives slice_llr with
 * those slices unknown.  Labels cover every bit pattern, so both sums keep a
 * label and the result is finite for any priors other than NaN (NaN in gives
 * NaN out).  Weights whose linear form underflows take the log-domain pass.
 * prior_llr: device fp32 [m_bits][n] (only rows in prior_mask are read; may
 * be NULL when prior_mask == 0).  Requires known_mask, prior_mask < 2^m_bits,
 * disjoint, and neither containing j; otherwise as slice_llr.               */
cvr_status slice_llr_prior(const double* x, int64_t n, double sigma_n, const double* thresholds,
                           int32_t m_bits, int32_t labelling, int32_t j, uint32_t known_mask,
                           const uint8_t* slices, uint32_t prior_mask, const float* prior_llr,
                           int32_t out_dtype, void* llr_out, void* stream);

/* Hard soft-information: Alice's LLR for slice j when she treats her own
 * quantised bit as the output of a binary symmetric channel with crossover p
 * (the bit error ratio p_j estimated in Sec. II Step 4):
 *   L_j = (1 - 2 a_j) ln((1 - p) / p),
 * a_j = bit j of the label of x under the same quantiser as slice_quantize
 * (thresholds, labelling).  x: device fp64 [n]; llr_out: device [n] of
 * out_dtype (CVR_F32 or CVR_F64).  Requires 0 < p < 1 and 0 <= j < m_bits;
 * n = 0 is a no-op.                                                          */
cvr_status slice_llr_bsc(const double* x, int64_t n, const double* thresholds, int32_t m_bits,
                         int32_t labelling, int32_t j, double p, int32_t out_dtype, void* llr_out,
                         void* stream);

/* Multistage decoding of consecutive slices (Sec. III-B steps 4-5): the LLR of
 * slice j exactly as slice_llr computes it (llr_out), and in the same pass
 * the LLR of slice j+1 under known_mask | (1 << j) for bit j = 0 (next_if0)
 * and bit j = 1 (next_if1).  The interval probabilities slice j+1 needs are
 * among those visited for slice j, and each conditional LLR is summed in the
 * order slice_llr(j+1, ...) uses, so both equal slice_llr with that bit held
 * known, bit for bit.  Once slice j is decoded, slice_llr_choose picks
 * per sample.  Requires 0 <= j, j + 1 < m_bits, bits j and j+1 clear in
 * known_mask; outputs: device [n] of out_dtype; otherwise as slice_llr.     */
cvr_status slice_llr_next(const double* x, int64_t n, double sigma_n, const double* thresholds,
                          int32_t m_bits, int32_t labelling, int32_t j, uint32_t known_mask,
                          const uint8_t* slices, int32_t out_dtype, void* llr_out, void* next_if0,
                          void* next_if1, void* stream);

/* llr_out[i] = (bits[i] & 1) ? llr_if1[i] : llr_if0[i] for i < n; the three
 * LLR arrays are device [n] of dtype (CVR_F32 or CVR_F64), bits device uint8
 * [n] (e.g. the decoded slice j).  n = 0 is a no-op.                        */
cvr_status slice_llr_choose(const void* llr_if0, const void* llr_if1, const uint8_t* bits, int64_t n,
                            int32_t dtype, void* llr_out, void* stream);

/* ------------------------------------------------------------------------- */
/* Syndromes                                                                  */
/* ------------------------------------------------------------------------- */
/* s = H b mod 2 for F frames of one code (Sec. II Step 5; Sec. III-B steps
 * 2-3), and the number of checks where it differs from a reference syndrome
 * (failure detection).  bits: device uint8 [F][n]; syndrome: device uint8
 * [F][m] or NULL (= all zero); syndrome_out: device uint8 [F][m] or NULL;
 * n_unsat: device int32 [F] or NULL (overwritten, not accumulated).
 * F = 0 is a no-op.                                                          */
cvr_status syndrome_check(cvr_code_t code, int32_t F, const uint8_t* bits,
                          const uint8_t* syndrome, uint8_t* syndrome_out,
                          int32_t* n_unsat, void* stream);

/* ------------------------------------------------------------------------- */
/* Batched belief-propagation decoding of sub-blocks                          */
/* ------------------------------------------------------------------------- */
/* A ragged batch: frame f uses codes[code_idx] and occupies variables
 * [vn_offset, vn_offset + n) of the LLR/bit arrays and checks
 * [chk_offset, chk_offset + m) of the syndrome array (Sec. III-A: N_d
 * independent decoders, possibly of different codes).  Frames must not
 * overlap.  The batch handle owns a device copy of the frame table and the
 * work lists; the codes must outlive it.                                     */
typedef struct {
    int32_t code_idx;
    int32_t reserved;
    int64_t vn_offset;
    int64_t chk_offset;
} cvr_frame;

typedef struct cvr_batch_s* cvr_batch_t;

cvr_status cvr_batch_create(const cvr_code_t* codes, int32_t n_codes, const cvr_frame* frames,
                            int32_t F, cvr_batch_t* out);
/* Extent of the batch: required lengths of the variable and check arrays. */
cvr_status cvr_batch_info(cvr_batch_t batch, int32_t* F, int64_t* total_n, int64_t* total_m,
                          int64_t* total_edges);
cvr_status cvr_batch_destroy(cvr_batch_t batch);

/* Decoder parameters.  The paper fixes only "belief propagation" (Sec.
 * III-C); the variant, schedule, stopping rule and precision are these:
 *  algo      CVR_SP: sum-product, c2v = (1-2s_c) prod sign * phi(sum phi|v2c|),
 *                    phi(x) = -ln tanh(x/2), v2c clamped to +-msg_clamp first;
 *            CVR_NMS: normalized min-sum, c2v = w (1-2s_c) prod sign * min|v2c|,
 *                    w = weights[t][edge_type] or alpha when weights is NULL.
 *  Flooding schedule (every check, then every variable, per iteration) unless
 *  schedule is CVR_SCHED_LAYERED.  The syndrome of the hard decisions is
 *  tested before the first iteration and after each one; a frame stops at the
 *  first success when early_stop != 0, and after max_iter iterations otherwise.
 *  math      CVR_F32 or CVR_F64: arithmetic precision and the dtype of llr,
 *            llr_post_out and trace.
 *  store     precision of the stored check-to-variable messages: CVR_F64
 *            (math must be F64), CVR_F32, or CVR_F16 (round to nearest even,
 *            saturating at +-65504; math F32).
 *  weights   device fp32 [max_iter][n_types] or NULL.
 *  trace     device [max_iter + 1][total_n] of the math dtype, or NULL: the
 *            posteriors after every iteration (row 0 = channel LLRs); rows past
 *            a frame's stop are not written for that frame.
 *  schedule  how the flooding iterations are launched (results are identical):
 *            CVR_SCHED_PASSES: two kernel launches per iteration over all
 *            frames (any code); CVR_SCHED_PERSISTENT: one persistent launch in
 *            which each workgroup iterates whole frames to their stop (QC codes
 *            with <= 2048 circulants, <= 512 block rows/columns and Z <= 65535, else
 *            CVR_EUNSUPPORTED); CVR_SCHED_GROUP: one launch with a workgroup
 *            per compute unit, in groups of workgroups on one XCD (accelerator
 *            complex die: its compute units share an L2 cache), each group
 *            decoding one frame at a time with barriers between the passes (the
 *            same codes as persistent; every compute unit must be free for the
 *            launch, else a barrier gives up after 0.2 s and every frame of
 *            the decode is reported abandoned: iters_out = -1, ok_out = 0);
 *            CVR_SCHED_AUTO: for the codes of the
 *            persistent schedule, persistent when the batch has at least one
 *            frame per compute unit and group below that; passes otherwise.
 *            CVR_SCHED_LAYERED is another message-passing order, so its
 *            results differ from flooding: the layered (row-serial) schedule
 *            over the block rows of a QC code (Sec. III-C names belief
 *            propagation without fixing a schedule).  Iteration t updates block
 *            row 0, 1, ..., mb-1 in turn; row k of block row i forms
 *            x_e = L[v] - c2v_e for its edges, computes c2v_e by the check rule
 *            (weights of iteration t) and sets L[v] = x_e + c2v_e with the
 *            stored c2v_e, so later block rows see the updated L.  L starts
 *            as the channel LLRs; the syndrome test, stop rule and outputs are
 *            those of flooding.  One workgroup decodes a frame (the codes of
 *            the persistent schedule whose decision bits fit in LDS beside the
 *            code tables, else CVR_EUNSUPPORTED; Bob's syndrome bits go to the
 *            workspace when they do not fit as well); consecutive
 *            block rows with no block column in common run in one step (their
 *            updates commute, so results equal one block row at a time);
 *            wg_threads may be 0 (= 512), 256, 512 or 1024 and lds_cache_kb
 *            applies; min_waves and group_wgs are ignored.
 *  wg_threads, min_waves  tuning knobs of the persistent decoder that do
 *            not change results: workgroup size 512 or 1024 (0 = 512);
 *            min_waves 8 compiles for 8 resident waves per SIMD, 0 lets the
 *            compiler choose.  1024 threads with min_waves 0 (one workgroup
 *            per compute unit) give each thread 4 rows of a block row per step
 *            when Z % 256 == 0, 2 when Z % 128 == 0.  Binary64 math and
 *            batches with a check row of more than 8 edges always run 512
 *            threads.  The group schedule runs 1024 threads (512 in those
 *            cases) and takes min_waves too: 8 puts two workgroups on each
 *            compute unit.
 *  lds_cache_kb  posteriors of the highest-degree block columns that the
 *            persistent decoder keeps in LDS (results unchanged): 0 = as much
 *            as fits without fewer resident workgroups, -1 = none, > 0 = that
 *            many KiB (capped by the LDS size).
 *  group_wgs workgroups per frame of the group schedule (results unchanged):
 *            0 = the workgroups an XCD holds divided by its frames, at least
 *            1; capped by the workgroups an XCD holds.                        */
enum { CVR_SCHED_AUTO = 0, CVR_SCHED_PASSES = 1, CVR_SCHED_PERSISTENT = 2, CVR_SCHED_GROUP = 3,
       CVR_SCHED_LAYERED = 4 };

typedef struct {
    int32_t algo;
    int32_t max_iter;          /* >= 0 */
    int32_t early_stop;
    int32_t math;
    int32_t store;
    float alpha;
    float msg_clamp;           /* > 0; SP only */
    int32_t schedule;
    int32_t wg_threads;
    int32_t min_waves;
    int32_t lds_cache_kb;
    int32_t group_wgs;
    const float* weights;
    void* trace;
} cvr_decode_params;

/* Bytes of device workspace ldpc_decode_batch needs for this batch/params
 * (messages, posteriors, per-frame flags and counters; on the layered
 * schedule also room for Bob's syndrome bits of frames whose decision and
 * syndrome bits do not fit in LDS together). */
cvr_status cvr_decode_workspace_size(cvr_batch_t batch, const cvr_decode_params* params,
                                     size_t* bytes);

/* Decodes every frame of the batch.
 *  llr:          device [total_n] channel LLRs (math dtype);
 *  syndrome:     device uint8 [total_m] Bob's syndromes, or NULL (all zero);
 *  bits_out:     device uint8 [total_n] hard decisions at the stop;
 *  llr_post_out: device [total_n] posteriors at the stop (math dtype) or NULL;
 *  iters_out:    device int32 [F] iteration at which the frame stopped, or -1
 *                when the decode was abandoned (a group barrier gave up, see
 *                CVR_SCHED_GROUP): the frame's other outputs are then invalid;
 *  ok_out:       device uint8 [F] 1 iff the syndrome was satisfied at the stop;
 *  workspace:    device, >= cvr_decode_workspace_size bytes, 256-byte aligned.
 * Non-finite LLRs are allowed.  A check touching a NaN posterior counts as
 * unsatisfied, so a frame fed a NaN LLR ends with ok = 0.                   */
cvr_status ldpc_decode_batch(cvr_batch_t batch, const cvr_decode_params* params,
                             const void* llr, const uint8_t* syndrome, uint8_t* bits_out,
                             void* llr_post_out, int32_t* iters_out, uint8_t* ok_out,
                             void* workspace, size_t ws_bytes, void* stream);

/* The same decode for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * no workspace argument; the workspace is a static device array of
 * CVR_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until the
 * process ends.  Calls no hipMalloc / hipFree (the batch and codes are
 * created beforehand, as for ldpc_decode_batch).  Same arguments, outputs and
 * results as ldpc_decode_batch.  A batch whose cvr_decode_workspace_size
 * exceeds CVR_NOALLOC_SCRATCH_BYTES returns CVR_ENOMEM before anything is
 * enqueued.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (two streams, or two host threads, without ordering
 * between them) race and give undefined results; calls in one stream are
 * ordered and safe.  Each call reinitialises what the decode reads from the
 * array, so no clearing is needed between calls.                           */
#define CVR_NOALLOC_SCRATCH_BYTES (64u << 20)
cvr_status ldpc_decode_batch_noalloc(cvr_batch_t batch, const cvr_decode_params* params,
                                     const void* llr, const uint8_t* syndrome, uint8_t* bits_out,
                                     void* llr_post_out, int32_t* iters_out, uint8_t* ok_out,
                                     void* stream);

/* ------------------------------------------------------------------------- */
/* Differentiable unrolled normalized min-sum (learning per-iteration,        */
/* per-edge-type scales)                                                      */
/* ------------------------------------------------------------------------- */
/* T iterations of binary32 min-sum with weights w[t][type] (no early stop,
 * fp32 messages) on a QC batch (as the persistent schedule requires, at most
 * 4 edge types, every check of degree >= 2).  The forward posteriors equal
 * those of ldpc_decode_batch(CVR_NMS, F32/F32, weights, early_stop = 0).
 * The messages c2v(t) at t = 0, K, 2K, ... (K = ckpt_every) are checkpointed;
 * the backward pass recomputes each K-iteration segment from its checkpoint
 * and runs the adjoint through it: derivatives flow through the minimum to
 * its lowest-index minimiser, |x| has derivative sign(x) (sign(0) = +1) and
 * sign products are constant.  The weight gradient is reduced in a fixed
 * order (bit-identical across runs on one device).
 *
 * nms_unrolled_sizes: ckpt_floats = floats of the checkpoint buffer; bytes of
 *   the forward and backward workspaces (any output pointer may be NULL).
 * nms_unrolled_fwd: weights device fp32 [T][n_types]; llr device fp32
 *   [total_n]; syndrome device uint8 [total_m] or NULL; llr_post_out device
 *   fp32 [total_n] = L_post(T); ckpt device fp32 [ckpt_floats] (written).
 * nms_unrolled_bwd: ckpt as written by the forward with the same arguments;
 *   dloss_dpost device fp32 [total_n]; dweights device fp32 [T][n_types]
 *   (overwritten); dllr device fp32 [total_n] or NULL (overwritten).        */
cvr_status nms_unrolled_sizes(cvr_batch_t batch, int32_t T, int32_t ckpt_every, size_t* ckpt_floats,
                              size_t* fwd_workspace, size_t* bwd_workspace);
cvr_status nms_unrolled_fwd(cvr_batch_t batch, int32_t T, int32_t ckpt_every, const float* weights,
                            const float* llr, const uint8_t* syndrome, float* llr_post_out, float* ckpt,
                            void* workspace, size_t ws_bytes, void* stream);
cvr_status nms_unrolled_bwd(cvr_batch_t batch, int32_t T, int32_t ckpt_every, const float* weights,
                            const float* llr, const uint8_t* syndrome, const float* ckpt,
                            const float* dloss_dpost, float* dweights, float* dllr, void* workspace,
                            size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------- */
/* Launch timing                                                              */
/* ------------------------------------------------------------------------- */
/* Kernel kinds reported by cvr_profile_read. */
enum {
    CVR_PROF_QUANTIZE = 0,     /* slice_quantize                                  */
    CVR_PROF_LLR = 1,          /* slice_llr                                       */
    CVR_PROF_SYNDROME = 2,     /* syndrome_check                                  */
    CVR_PROF_CHECK = 3,        /* decoder check-node pass (one per iteration)     */
    CVR_PROF_VAR = 4,          /* decoder variable-node pass (one per iteration)  */
    CVR_PROF_DEC_SETUP = 5,    /* decoder set-up and output passes                */
    CVR_PROF_FRAMES = 6,       /* persistent decoder (whole decode in one launch) */
    CVR_PROF_ADJOINT = 7       /* nms_unrolled_bwd (adjoint of unrolled min-sum)  */
};

/* on != 0: every later launch of the library is bracketed by two HIP events on
 * its stream (process-wide switch; adds two event records per launch). */
cvr_status cvr_profile_enable(int32_t on);

/* Waits for the recorded events and returns the summed duration (ms) and the
 * number of launches of one kind since the last reset; reset != 0 clears them. */
cvr_status cvr_profile_read(int32_t kind, double* total_ms, int64_t* launches, int32_t reset);

/* ------------------------------------------------------------------------- */
/* Testing hook                                                               */
/* ------------------------------------------------------------------------- */
/* Bounds every wait at a barrier of the group schedule (CVR_SCHED_GROUP) to
 * `ticks` of the 100 MHz device wall clock, for later launches of this
 * process; the default is 20,000,000 (0.2 s).  With 0 a barrier that is not
 * complete when a workgroup arrives gives up at once: the launch still ends,
 * and every frame of that decode is reported abandoned, iters = -1 and
 * ok = 0 (the path a barrier takes when a group's workgroups are not all
 * resident).  For tests of that failure path.  ticks > 1e10 returns CVR_EINVAL. */
cvr_status cvr_debug_group_wait_ticks(uint64_t ticks);

#ifdef __cplusplus
}
#endif
#endif /* CVQKD_RECON_H */
