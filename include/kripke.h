/*
 * kripke.h -- C ABI of the MI355X Kripke census library (libkripke.so).
 *
 * The library evaluates modal formulas over every labelled Kripke frame of a
 * given size and every valuation (Section 3: world sets as bitmasks, BOX as
 * successor-mask containment, DIA as intersection, Lemma 1 and Theorem 1) on
 * gfx950 GPUs, and reports per formula the failure count and the first
 * countermodel (Algorithm 1, Definition 1).  It also searches frame lists for
 * the first model separating two formulas (Definition 2, Proposition 5).
 *
 * Conventions shared by every entry point
 *   - Status: 0 on success, a negative KRIPKE_E* code on failure.  On failure
 *     nothing has been enqueued; kripke_last_error() gives a message
 *     (thread-local, valid until the next call on the same thread).
 *   - Formula programs are postfix bytecode, one byte per node, so the byte
 *     length equals the node count |phi| of Section 2:
 *       0 TOP  1 BOT  2+i VAR p_i (i < 4)  6 NOT  7 AND  8 OR  9 IMP
 *       10 BOX  11 DIA  12 IFF (biconditional; used for Proposition 5)
 *     A batch is CSR-packed: `code` holds the programs back to back and
 *     `offsets[b] .. offsets[b+1]` delimits program b (offsets has B+1 entries,
 *     offsets[0] = 0).  code/offsets are HOST pointers; the library validates
 *     them synchronously and copies what it needs before returning.
 *   - Frame index f on n worlds (a labelled frame, Section 3): bit (w*n + v)
 *     of f is set iff w R v; successor mask succ[w] = (f >> n*w) & (2^n - 1).
 *   - Valuation index val for k variables: bit (i*n + w) of val is set iff
 *     p_i holds at world w; valuations run over [0, 2^(k*n)).
 *   - A countermodel key packs (frame, valuation, world) lexicographically:
 *       key = frame << (k*n + 4) | val << 4 | world
 *     so the numerically least key is the lexicographically first
 *     countermodel.  KRIPKE_NO_KEY (all ones) means none was found.  For
 *     filtered classes the frame field is the raw frame index above, not a
 *     rank within the class.  For split searches the frame field is the
 *     position in the caller's frame list.
 *   - Output and frame buffers are DEVICE pointers owned by the caller (for
 *     example torch tensors).  Every launch is asynchronous on the HIP stream
 *     passed as `stream` (NULL = the null stream); results are valid once
 *     the stream has been synchronised.  The library owns only its plans and
 *     internal workspace.
 *   - Calls that share a plan must not overlap; distinct plans may run
 *     concurrently on distinct streams.
 */
#ifndef KRIPKE_H
#define KRIPKE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KRIPKE_OK 0
#define KRIPKE_EINVAL (-1)   /* null pointer, empty batch, bad class/flag      */
#define KRIPKE_EPROGRAM (-2) /* unknown opcode, stack under/overflow, var >= k */
#define KRIPKE_ELIMIT (-3)   /* n, nvars, key width or program length limits  */
#define KRIPKE_EHIP (-4)     /* a HIP runtime call failed                      */
#define KRIPKE_ENOMEM (-5)   /* device or host allocation failed               */
#define KRIPKE_EINTERNAL (-6) /* an internal consistency check failed          */

#define KRIPKE_NO_KEY UINT64_MAX

/* Frame classes of Section 2; each is contained in the previous one. */
typedef enum {
  KRIPKE_K = 0,  /* all frames                      */
  KRIPKE_T = 1,  /* reflexive                       */
  KRIPKE_S4 = 2, /* reflexive and transitive        */
  KRIPKE_S5 = 3  /* equivalence relations           */
} kripke_class;

/* Per-formula result of one (class, n) layer (Algorithm 1's FAIL and FIRST,
 * 16 bytes as in the paper's fused reduction). */
typedef struct {
  uint64_t first_key;  /* least countermodel key, or KRIPKE_NO_KEY (valid) */
  uint64_t fail_count; /* number of (frame in class, valuation) pairs with a
                          falsifying world                                 */
} kripke_census_result;

/* kripke_census_range flags */
#define KRIPKE_COUNT 0u  /* exact fail_count and first_key                       */
#define KRIPKE_DECIDE 1u /* first_key only; scanning stops at the first
                            countermodel, fail_count is left undefined           */

/* Limits: 1 <= n <= 6 for census; n*n + nvars*n + 4 <= 64; nvars <= 4;
 * program length 1..255 nodes. */

/*
 * kripke_census -- census of a formula batch over every frame on exactly n
 * worlds in class `cls` and every valuation of p_0..p_{nvars-1}
 * (Algorithm 1 over one (class, n) layer; Theorem 1 gives exactness).
 * d_out: device array of nformulas results, overwritten.
 * n <= 5 (use kripke_census_range for n = 6).
 */
int kripke_census(const uint8_t *code, const uint32_t *offsets, uint32_t nformulas, uint32_t n,
                  uint32_t cls, uint32_t nvars, kripke_census_result *d_out, void *stream);

/*
 * kripke_census_range -- the same census restricted to raw frame indices in
 * [frame_begin, frame_end) (frames outside the class are skipped), so a
 * census can be sliced, checkpointed and resumed: merging slices with
 * min(first_key) and sum(fail_count) equals the one-shot result.  This is the
 * scan of Section 5's bounded decision (Theorem 2) restricted to part of one
 * layer; with KRIPKE_DECIDE it stops at the first countermodel, the witness
 * Theorem 2 (2) asks for.
 * flags: KRIPKE_COUNT or KRIPKE_DECIDE.  1 <= n <= 6 (S4 and S5: n <= 5).
 * d_out: device array of nformulas results, overwritten.
 */
int kripke_census_range(const uint8_t *code, const uint32_t *offsets, uint32_t nformulas,
                        uint32_t n, uint32_t cls, uint32_t nvars, uint64_t frame_begin,
                        uint64_t frame_end, uint32_t flags, kripke_census_result *d_out,
                        void *stream);

/*
 * kripke_census_range_static -- kripke_census_range for callers that cannot
 * allocate device memory (tight serving loops, hosts that forbid device
 * allocation during a run): same arguments, same results, but no
 * hipMalloc/hipFree or allocating library call is made.  Its working
 * memory (the compiled programs, their launch order and two work-queue
 * counters) lives in one fixed static device array of about 1.1 MB per GPU,
 * held from the first call on that GPU until the process ends.
 * Limits beyond kripke_census_range's: classes K and T only (S4 and S5 need
 * the frame lists the library allocates; KRIPKE_EINVAL), at most
 * KRIPKE_STATIC_MAX_FORMULAS formulas and KRIPKE_STATIC_MAX_CODE bytes of
 * compiled programs (each program compiles to at most 2 * length + 2 micro-ops,
 * padded to 8 bytes; KRIPKE_ELIMIT).
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on the same GPU (on different streams or threads) race and give undefined
 * results; calls serialised on one stream are safe.  The call waits for its
 * host-to-device copies (a stream synchronisation) before enqueuing kernels,
 * so it cannot be recorded into a graph under stream capture.
 */
#define KRIPKE_STATIC_MAX_FORMULAS 8192u
#define KRIPKE_STATIC_MAX_CODE (1u << 20)
int kripke_census_range_static(const uint8_t *code, const uint32_t *offsets,
                               uint32_t nformulas, uint32_t n, uint32_t cls, uint32_t nvars,
                               uint64_t frame_begin, uint64_t frame_end, uint32_t flags,
                               kripke_census_result *d_out, void *stream);

/*
 * kripke_frame_validity -- per-frame validity maps (Section 10: Val_N(phi),
 * the set of frames on which phi holds at every world under every valuation,
 * the input of frame-correspondence recovery).  For every formula and every
 * frame index f in [0, 2^(n*n)) (class K), bit f % 32 of word f / 32 of row
 * i is 1 iff formula i has no countermodel on frame f.
 * d_bits: DEVICE uint32[nformulas][ceil(2^(n*n) / 32)], overwritten.
 * Limits: 4 <= n <= 5, n * nvars <= 11; otherwise KRIPKE_ELIMIT.
 */
int kripke_frame_validity(const uint8_t *code, const uint32_t *offsets, uint32_t nformulas,
                          uint32_t n, uint32_t nvars, uint32_t *d_bits, void *stream);

/*
 * kripke_split -- first model separating phi and psi (Definition 2; by
 * Proposition 5 a countermodel of phi <-> psi) over a caller-owned device
 * frame list d_frames (uint32 succ[nframes][n], row-major, bit v of
 * succ[w] set iff w R v), scanning positions in order, then valuations, then
 * worlds.  *d_first_key (device, 1 value) receives
 * position << (nvars*n + 4) | val << 4 | world, or KRIPKE_NO_KEY.
 * Limits: 1 <= n <= 16; nvars <= 4, nvars <= 3 for n >= 7, and
 * nvars * n <= 24 for n >= 9; the key must fit 64 bits (bits for the
 * position + nvars*n + 4 <= 64); otherwise KRIPKE_ELIMIT.  Frames of 11 or
 * more worlds (and of 9 or 10 worlds with two or more variables) run on a
 * per-lane world-mask kernel, the others on the bit-sliced kernels (six-world
 * lists with two variables: two list frames per block; each block is decoded
 * once for a group of up to four pairs).  For comparisons, the environment
 * variables KRIPKE_SPLIT_GENERIC=1 (per-lane-frame kernel),
 * KRIPKE_SPLIT_WORLDMASK=1 (world-mask kernel at any size),
 * KRIPKE_SPLIT_ONE_FRAME=1 (one list frame per block) and
 * KRIPKE_LIST_GROUP=1..4 (pairs per group of the list kernels) select
 * other kernels; every kernel returns the same keys.
 */
int kripke_split(const uint8_t *phi, uint32_t len_phi, const uint8_t *psi, uint32_t len_psi,
                 const uint32_t *d_frames, uint64_t nframes, uint32_t n, uint32_t nvars,
                 uint64_t *d_first_key, void *stream);

/*
 * kripke_split_batch -- kripke_split for npairs pairs at once.  The CSR batch
 * holds 2*npairs programs: program 2j is phi_j and 2j+1 is psi_j.
 * d_first_key: device uint64[npairs].
 */
int kripke_split_batch(const uint8_t *code, const uint32_t *offsets, uint32_t npairs,
                       const uint32_t *d_frames, uint64_t nframes, uint32_t n, uint32_t nvars,
                       uint64_t *d_first_key, void *stream);

/* Key and frame codecs (host-only, no device work): the successor-mask
 * encoding of a labelled frame and the packed (frame, valuation, world)
 * countermodel of Section 3's bitmask model (world sets as n-bit masks). */
void kripke_key_decode(uint64_t key, uint32_t n, uint32_t nvars, uint64_t *frame,
                       uint64_t *valuation, uint32_t *world);
void kripke_frame_decode(uint64_t frame, uint32_t n, uint32_t *succ /* [n] */);

/*
 * Plans: a batched census of one formula batch over all frames on n worlds
 * for every class in class_mask (bit c = kripke_class c) in ONE persistent
 * launch that enumerates K frames once and reduces each frame into every
 * class containing it, captured in a hipGraph on first launch and replayed
 * afterwards.  This is Section 4's fused corpus scan (the whole batch in one
 * kernel with per-formula reductions, compared there with separate launches
 * per formula).  n <= 5, nformulas >= 1; the plan owns its device copies and
 * must be destroyed with kripke_plan_destroy.  tune_cache: path of a JSON file of autotuned tile choices
 * (frame sets per lane, work items per wave).  NULL uses the defaults; with
 * a path, a cached choice for this device, n, nvars and batch is reused, and
 * otherwise every candidate is timed on a slice of the frames at creation
 * (the per-formula form below: on the first 256 formulas of the batch)
 * and the winner is appended to the file.  With the environment variable
 * KRIPKE_TUNE_LOG=1 each candidate's time is printed to stderr.
 * d_out: device array [4][nformulas] (class-major); rows of classes not in
 * class_mask are left untouched.
 * Every tile candidate the autotuner times must give identical results on
 * its frame slice; otherwise creation fails with KRIPKE_EINTERNAL.
 * KRIPKE_PLAN_PLAIN in class_mask selects an unbatched baseline instead, no
 * graph -- the "separate launches" form the batched plan is compared with:
 * with tune_cache NULL, the per-class kernels launched once per formula and
 * class with default tiles; with a tune_cache (class_mask 0xF), the fused
 * all-class kernel launched once per formula with tiles autotuned for that
 * form (cached under its own key).
 */
#define KRIPKE_PLAN_PLAIN 0x10u
int kripke_plan_create(const uint8_t *code, const uint32_t *offsets, uint32_t nformulas,
                       uint32_t n, uint32_t class_mask, uint32_t nvars, const char *tune_cache,
                       void **plan);
int kripke_plan_launch(void *plan, kripke_census_result *d_out, void *stream);
int kripke_plan_destroy(void *plan);

/*
 * kripke_program_stats -- host-only introspection of the compiled programs.
 * The library compiles every formula into an equivalent program by exact
 * rewrites (constant folding, negation normal form, operand ordering); this
 * reports, per formula, the work one evaluation of the compiled program
 * performs, in the terms of Proposition 2's cost bound (Boolean and modal
 * operators).  stats: int32[nformulas][6] =
 *   {modal ops, binary ops, leaf loads, stack saves, stack slots, constant}
 * where constant is 1/0 if the formula folds to TOP/BOT, else -1.
 */
int kripke_program_stats(const uint8_t *code, const uint32_t *offsets, uint32_t nformulas,
                         uint32_t nvars, int32_t *stats);

/*
 * kripke_calibrate_int32 -- measured rate of plain 32-bit bitwise vector
 * instructions on the current device (lane-operations per second), the
 * ceiling the evaluator is compared against (Section 8's integer calibration:
 * dependent XOR/AND/OR chains).  Runs synchronously (about
 * 50 ms) on `stream`.
 */
int kripke_calibrate_int32(double *lane_ops_per_s, void *stream);

/* ------------------------------------------------------------------
 * Learned pair proposal (candidate generation and ranking before exact
 * verification; the paper's analogue is representation-guided retrieval in
 * Section 9 followed by exhaustive rescans).
 * ------------------------------------------------------------------ */

/*
 * kripke_signatures -- truth bits of each formula at a list of pointed
 * models (Section 2 satisfaction), used as a semantic signature.
 * samples: HOST array of nsamples packed models
 *   n << 60 | frame << 24 | valuation << 4 | world   (1 <= n <= 3),
 * nsamples a multiple of 64, each aligned run of 64 samples with one n.
 * d_sig: DEVICE uint64[nformulas][nsamples / 64]; bit s%64 of word s/64 of
 * row i is 1 iff formula i holds at sample s.
 */
int kripke_signatures(const uint8_t *code, const uint32_t *offsets, uint32_t nformulas,
                      uint32_t nvars, const uint64_t *samples, uint32_t nsamples,
                      uint64_t *d_sig, void *stream);

/*
 * kripke_knn_pairs -- candidate pairs: for every formula its k nearest
 * formulas by signature Hamming distance (ties to the smaller index), as
 * unordered pairs (i < j) packed i << 32 | j, deduplicated and in canonical
 * (i, j) order.  d_sig: DEVICE [nformulas][words] (words*64 <= 8192,
 * nformulas <= 16384, 0 < k < nformulas).  d_pairs: DEVICE uint64 capacity
 * nformulas*k; d_npairs: DEVICE uint64 (count written).
 */
int kripke_knn_pairs(const uint64_t *d_sig, uint32_t nformulas, uint32_t words, uint32_t k,
                     uint64_t *d_pairs, uint64_t *d_npairs, void *stream);

/* Signature Hamming distance of each pair (d_pairs packed as above). */
int kripke_pair_hamming(const uint64_t *d_sig, uint32_t words, const uint64_t *d_pairs,
                        uint64_t npairs, uint32_t *d_dist, void *stream);

/*
 * kripke_select_top -- indices of the `budget` largest of n float scores,
 * largest first, equal scores in increasing index order.  All DEVICE
 * pointers; d_idx holds min(budget, n) uint64.
 */
int kripke_select_top(const float *d_scores, uint64_t n, uint64_t budget, uint64_t *d_idx,
                      void *stream);

/*
 * Pair-scoring MLP (the learned proposal; it stands in for the representation
 * layouts of Section 9's retrieval): input
 * [sig_a XOR sig_b, sig_a AND sig_b] of two 4,096-bit signatures (8,192
 * values in {0,1}) -> 512 -> 256 -> 1, ReLU; BF16 weights and activations as
 * matrix-core operands, FP32 accumulation, FP32 master weights, Adam.
 * Parameters (FP32, 4,326,401 values, in this order): W1 [512][8192],
 * b1 [512], W2 [256][512], b2 [256], w3 [256], b3 [1]; W is (out x in).
 * Pairs are DEVICE uint64 packed a << 32 | b (row indices of d_sig); d_sig
 * is DEVICE uint64 [rows][words] with words = 64.
 */
int kripke_mlp_create(uint64_t seed, uint32_t max_batch, void **mlp);
int kripke_mlp_destroy(void *mlp);
/* Host copies of the FP32 parameters / gradients (4,326,401 floats). */
int kripke_mlp_get_params(void *mlp, float *params);
/* Replace the parameters (and reset the Adam moments and step count). */
int kripke_mlp_set_params(void *mlp, const float *params);
int kripke_mlp_get_grads(void *mlp, float *grads);
/* Logits of npairs pairs (any count; processed in chunks of max_batch). */
int kripke_mlp_forward(void *mlp, const uint64_t *d_sig, uint32_t words, const uint64_t *d_pairs,
                       uint64_t npairs, float *d_logits, void *stream);
/* Mean BCE-with-logits loss (positive weight pos_weight) of one batch of m
 * labelled pairs (m a multiple of 64, m <= max_batch) and all parameter
 * gradients, kept inside the handle.  d_labels: DEVICE float[m] in {0,1};
 * d_loss: DEVICE float[1]. */
int kripke_mlp_gradients(void *mlp, const uint64_t *d_sig, uint32_t words,
                         const uint64_t *d_pairs, const float *d_labels, uint32_t m,
                         float pos_weight, float *d_loss, void *stream);
/* One Adam step (bias-corrected) from the gradients of the last
 * kripke_mlp_gradients call; refreshes the BF16 working copies. */
int kripke_mlp_adam_step(void *mlp, float lr, float beta1, float beta2, float eps, void *stream);

/* Message for the last failure on this thread ("" if none). */
const char *kripke_last_error(void);

/* Library version (major * 10000 + minor * 100 + patch). */
int kripke_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KRIPKE_H */
