/*
 * ymine -- comparable-corpus sentence miner for AMD Instinct MI355X (gfx950).
 *
 * C ABI of the GPU library (libymine.so).  The operation is the improved
 * Yalign-style mining of Section 4 of Wolk & Marasek, "Tuned and
 * GPU-accelerated parallel data mining from comparable corpora"
 * (arXiv:1509.08639): for every comparable document pair, score every source
 * sentence against every target sentence with a classifier whose confidence
 * is a probability, align the score matrix with Needleman-Wunsch (monotone
 * paths, a penalty per skipped sentence), and accept the matched sentence
 * pairs whose confidence reaches the threshold.
 *
 * Definitions (all arithmetic fixed so results are reproducible bit for bit):
 *   T(x)      set of target ids that lexicon entry x translates to
 *   X_i       union of T(x) over the tokens x of source sentence i (a_i tokens)
 *   m_t(i,j)  number of positions of target sentence j (b_j tokens) holding an
 *             id in X_i
 *   m_s(i,j)  number of positions q of source sentence i whose T(s_i[q]) meets
 *             the id set of target sentence j
 *   f1 = m_s/a_i, f2 = m_t/b_j, f3 = min(a_i,b_j)/max(a_i,b_j)  (float; x/0 = 0)
 *   z = ((w0 + w1*f1) + w2*f2) + w3*f3   (float, each op rounded, no FMA)
 *   S[i][j] = (float)(1 / (1 + exp(-(double)z)))
 *   H[0][0] = 0; H[i][0] = H[i-1][0] + g; H[0][j] = H[0][j-1] + g (float,
 *   repeated addition); H[i][j] = max of D = H[i-1][j-1] + S[i-1][j-1],
 *   U = H[i-1][j] + g, L = H[i][j-1] + g, ties resolved D > U > L.
 *   The traceback from (n, m) yields the path; every D move into (i+1, j+1)
 *   with S[i][j] >= threshold emits the pair (i, j).
 *
 * Conventions
 *   - Every call returns a ym_status; nothing aborts or throws across the ABI.
 *     On failure ym_last_error() (thread-local) describes the cause.
 *   - Inputs are borrowed for the duration of the call.  Objects returned
 *     through `out` pointers are owned by the caller and released with the
 *     matching *_free / *_destroy call.
 *   - Token ids are int32.  An id that is not a lexicon key (including any
 *     negative id) has no translations and never matches; this is exactly
 *     the definition above, since lexicon ids are >= 0.
 *   - Results are deterministic: the same inputs give the same bits on every
 *     run, launch shape and batch composition.
 */
#ifndef YMINE_H
#define YMINE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ym_status;
#define YM_OK 0
#define YM_EPENDING 1     /* ym_poll: request not finished yet */
#define YM_EINVAL (-1)    /* malformed argument (offsets, sizes, non-finite parameters) */
#define YM_ENOMEM (-2)    /* host or device allocation failed, or workspace too small */
#define YM_EDEVICE (-3)   /* a HIP runtime call failed */
#define YM_EBUDGET (-4)   /* request larger than the serving HBM budget */
#define YM_ECANCELLED (-5)/* request cancelled */
#define YM_ENOTFOUND (-6) /* unknown ticket */

/* Largest number of target ids one lexicon key may translate to. */
#define YM_MAX_FANOUT 255

/* Size limits of one document pair, checked by every entry point before any
 * work is enqueued (YM_EINVAL otherwise): at most 2^22 sentences per document
 * and fewer than 2^31 score slots, about n * (m + 63) for n >= 64 (the
 * similarity kernels address a pair's scores with 32-bit offsets; n = m =
 * 46,000 is about the largest square pair).  Host-only, needs no device:
 * YM_OK if a pair of n source and m target sentences is accepted. */
ym_status ym_check_pair(int64_t n, int64_t m);

typedef struct ym_ctx ym_ctx;
typedef struct ym_lexicon ym_lexicon;
typedef struct ym_server ym_server;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`.  `hbm_budget_bytes` bounds the
 * device memory the serving loop may reserve for requests (0: 80% of free
 * memory).  The context owns a device arena reused across calls. */
ym_status ym_create(int device, size_t hbm_budget_bytes, ym_ctx **out);
/* Destroy a context.  Stop its servers first; lexicons may be freed before
 * or after it. */
void ym_destroy(ym_ctx *ctx);

/* Message of the last failure on this thread; never NULL. */
const char *ym_last_error(void);

/* Library build string (for logs). */
const char *ym_version(void);

/* ------------------------------------------------------------------ lexicon */

/* Load a bilingual lexicon: entry e translates source id src_ids[e] to the
 * target ids tgt_ids[off[e] .. off[e+1]).  All ids must be >= 0 and
 * off[0] = 0, off non-decreasing; a key may repeat (its sets are merged) and
 * target ids may repeat (they are a set).  The lexicon is normalised on the
 * host, copied to HBM and stays resident until ym_lexicon_free (the
 * classifier's data are loaded once per session, Section 4).  In HBM it is a
 * hash table over the keys and, when every key is below 2^24, also a table of
 * 16 bytes per id up to the largest key (at most 256 MB), which makes the
 * per-batch translation of source tokens a direct read.
 * Errors: YM_EINVAL for negative ids, bad offsets or a key with more than
 * YM_MAX_FANOUT distinct targets; YM_ENOMEM / YM_EDEVICE. */
ym_status ym_lexicon_load(ym_ctx *ctx, const int32_t *src_ids, const int64_t *off, const int32_t *tgt_ids,
                          int64_t n_src, ym_lexicon **out);
void ym_lexicon_free(ym_lexicon *lex);
/* Number of distinct keys and of (key, target) pairs held. */
ym_status ym_lexicon_stats(const ym_lexicon *lex, int64_t *n_keys, int64_t *n_pairs, int32_t *max_fanout);

/* ------------------------------------------------------------- batch layout */

/* A batch of document pairs in packed ragged form (three-level CSR).
 * Pair p's source document is sentences [src_doc_off[p], src_doc_off[p+1]);
 * source sentence s is tokens src_tok[src_sent_off[s] .. src_sent_off[s+1]).
 * Likewise for the target side.  All offsets are int64, start at 0 and are
 * non-decreasing; n_src_sent = src_doc_off[n_pairs], n_src_tok =
 * src_sent_off[n_src_sent].  Empty documents and empty sentences are valid. */
typedef struct {
  int64_t n_pairs;
  const int64_t *src_doc_off;  /* [n_pairs + 1] */
  const int64_t *src_sent_off; /* [n_src_sent + 1] */
  const int32_t *src_tok;      /* [n_src_tok] */
  const int64_t *tgt_doc_off;  /* [n_pairs + 1] */
  const int64_t *tgt_sent_off; /* [n_tgt_sent + 1] */
  const int32_t *tgt_tok;      /* [n_tgt_tok] */
} ym_batch;

/* Method parameters: classifier weights w[0..3] (bias, f1, f2, f3), the
 * penalty per skipped sentence `gap` (Section 4, "Penalty") and the
 * confidence `threshold` (Section 4, "Threshold").  All must be finite. */
typedef struct {
  float w[4];
  float gap;
  float threshold;
} ym_params;

/* Host result (CSR by pair).  Pair p's accepted sentence pairs are entries
 * [pair_off[p], pair_off[p+1]) of src_idx / tgt_idx / score, in path order
 * (both indices strictly increasing).  align_score[p] = H[n][m]. */
typedef struct {
  int64_t n_pairs;
  int64_t n_out;
  int64_t *pair_off;  /* [n_pairs + 1] */
  int32_t *src_idx;   /* [n_out] */
  int32_t *tgt_idx;   /* [n_out] */
  float *score;       /* [n_out] */
  float *align_score; /* [n_pairs] */
} ym_result;

/* ------------------------------------------------------------ batch mining */

/* Mine a host-resident batch (Section 4: per document pair, the classifier
 * scores every sentence pair, the score matrix is aligned with
 * Needleman-Wunsch, and aligned pairs at or above the threshold are kept);
 * the result is allocated by the library
 * (ym_result_free).  Internally: copy to HBM, similarity kernel, NW kernel
 * with device traceback and threshold, device compaction, copy back.  Large
 * batches are processed in chunks that fit the context's arena.  All-or-
 * nothing: on error *out is NULL. */
ym_status ym_mine(ym_ctx *ctx, const ym_lexicon *lex, const ym_batch *batch, const ym_params *params,
                  ym_result **out);
void ym_result_free(ym_result *res);

/* Same, one kernel launch sequence per document pair, each synchronised
 * before the next (the plain per-pair GPU form, kept as the comparison
 * baseline).  Results are identical to ym_mine. */
ym_status ym_mine_per_pair(ym_ctx *ctx, const ym_lexicon *lex, const ym_batch *batch, const ym_params *params,
                           ym_result **out);

/* Device-resident form.  `batch` holds HOST pointers for src_doc_off and
 * tgt_doc_off (the pair table, [n_pairs+1] each) and DEVICE pointers for the
 * sentence offsets and tokens; n_src_tok / n_tgt_tok bound every token read.
 * Outputs are DEVICE arrays: pair_off [n_pairs+1], align_score [n_pairs],
 * src_idx / tgt_idx / score with room for ym_mine_device_capacity() entries.
 * `workspace` is a device buffer of `workspace_bytes` (at least
 * ym_mine_device_workspace_min(); more lets larger chunks run at once).
 * Work is enqueued on `stream` (a hipStream_t, NULL = default stream); the
 * call returns once it is enqueued.  Host-side validation covers the pair
 * table; device offsets are clamped into their arrays, so malformed device
 * offsets give undefined results but no out-of-bounds access. */
typedef struct {
  int64_t n_pairs;
  const int64_t *src_doc_off;  /* host */
  const int64_t *tgt_doc_off;  /* host */
  const int64_t *src_sent_off; /* device */
  const int32_t *src_tok;      /* device */
  const int64_t *tgt_sent_off; /* device */
  const int32_t *tgt_tok;      /* device */
  int64_t n_src_tok, n_tgt_tok;
} ym_device_batch;

typedef struct {
  int64_t *pair_off;  /* device [n_pairs + 1] */
  int32_t *src_idx;   /* device [capacity] */
  int32_t *tgt_idx;   /* device [capacity] */
  float *score;       /* device [capacity] */
  float *align_score; /* device [n_pairs] */
  int32_t *status;    /* device, one int32, may be NULL: 0, or YM_EDEVICE once any
                         pair of the call could not be completed on the device */
} ym_device_out;

/* Device failures of this form are reported on the device, since the call
 * returns before its work runs: a pair whose sweep gives up (a bounded wait of
 * the pipelined NW sweep of a pair of 448 or more source sentences ran past
 * its limit) gets align_score NaN and no accepted pairs, and *out->status is
 * set to YM_EDEVICE (the library clears it to 0 at the start of the call).
 * The host entry points read these themselves and return YM_EDEVICE; a served
 * request that fails this way fails alone with YM_EDEVICE. */

/* Output capacity: sum over pairs of min(n, m). */
int64_t ym_mine_device_capacity(const int64_t *src_doc_off, const int64_t *tgt_doc_off, int64_t n_pairs);
/* Workspace that lets the whole batch run as one chunk, and the minimum
 * (both include 16 bytes per source token for the resolved translations). */
size_t ym_mine_device_workspace(const int64_t *src_doc_off, const int64_t *tgt_doc_off, int64_t n_pairs,
                                int64_t n_src_tok);
size_t ym_mine_device_workspace_min(const int64_t *src_doc_off, const int64_t *tgt_doc_off, int64_t n_pairs,
                                    int64_t n_src_tok);

ym_status ym_mine_device(ym_ctx *ctx, const ym_lexicon *lex, const ym_device_batch *batch,
                         const ym_params *params, void *workspace, size_t workspace_bytes,
                         const ym_device_out *out, void *stream);

/* Allocation-free form of ym_mine_device, for callers that cannot allocate
 * device or pinned host memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same batch, parameters, outputs,
 * stream semantics and results as ym_mine_device; the workspace is instead a
 * static device array of YM_STATIC_SCRATCH_BYTES per device, which the library
 * holds from the first ym_create on that device until the process ends.  The
 * call makes no hipMalloc, hipHostMalloc or hipFree: the score table and the
 * pinned plan staging buffer are set up by ym_create, and the batch is split
 * into chunks whose plans fit that staging buffer.
 * Errors: as ym_mine_device, and YM_ENOMEM (before any work is enqueued) when
 * ym_mine_device_workspace_min() of the batch exceeds YM_STATIC_SCRATCH_BYTES,
 * that is when 16 bytes per source token plus the largest pair's workspace do
 * not fit.  Every call on one device shares that device's array, and a call
 * leaves its contents in place (nothing in it needs to start cleared): calls
 * whose work overlaps on one device -- from several threads or contexts, or on
 * streams that are not ordered one after the other -- race and give undefined
 * results.  Order them (one stream, or events) to use this form. */
#define YM_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
ym_status ym_mine_device_static(ym_ctx *ctx, const ym_lexicon *lex, const ym_device_batch *batch,
                                const ym_params *params, const ym_device_out *out, void *stream);

/* --------------------------------------------------- parity / debug entries */

/* Similarity kernel alone on a host batch (Section 4: the classifier's
 * confidence for each sentence pair, from lexicon-overlap and length
 * features): S, m_s, m_t of every pair, row-
 * major n x m, pairs back to back in batch order (sum of n*m entries each).
 * m_s / m_t may be NULL. */
ym_status ym_similarity(ym_ctx *ctx, const ym_lexicon *lex, const ym_batch *batch, const ym_params *params,
                        float *S, int32_t *m_s, int32_t *m_t);

/* NW kernel alone (Section 4: the alignment of a document pair's score
 * matrix with a gap penalty, then the threshold on the aligned pairs), fed
 * score matrices from the host: pair p has n[p] x m[p]
 * scores at S + sum_{q<p} n[q]*m[q].  Outputs: align_score [n_pairs];
 * moves (may be NULL): pair p's forward path as 'D'/'U'/'L' bytes at offset
 * sum_{q<p} (n[q]+m[q]) with n_moves[p] entries; *out: accepted pairs. */
ym_status ym_nw_align(ym_ctx *ctx, const float *S, const int32_t *n, const int32_t *m, int64_t n_pairs,
                      float gap, float threshold, float *align_score, char *moves, int32_t *n_moves,
                      ym_result **out);

/* -------------------------------------------------- tuning and bidirectional */

/* Parameter sweep for the tuned miner (Section 4: penalty and threshold can
 * be adjusted, and this work adds a tuning algorithm for them; Section 5:
 * the NWT variant).  Scores are computed once per chunk and reused for every
 * gap in gaps[0..n_gaps): one NW launch per chunk sweeps all of them (its
 * outputs and scratch are held once per gap), and every threshold in
 * taus[0..n_taus) is applied while counting.  For the reference
 * pairs given as CSR per document pair (truth_off [n_pairs+1], sentence index
 * pairs truth_src / truth_tgt), n_mined[g * n_taus + t] receives the number
 * of accepted pairs and n_correct[...] how many of them are reference pairs;
 * precision, recall and F1 follow (recall denominator: truth_off[n_pairs]). */
ym_status ym_tune(ym_ctx *ctx, const ym_lexicon *lex, const ym_batch *batch, const float w[4], const float *gaps,
                  int32_t n_gaps, const float *taus, int32_t n_taus, const int64_t *truth_off,
                  const int32_t *truth_src, const int32_t *truth_tgt, int64_t *n_mined, int64_t *n_correct);

/* The parameter choice of the tuned miner: the (gap, threshold) entry of a
 * sweep with the highest F1 against the reference pairs (the paper tunes
 * penalty and threshold but gives no objective; F1 is this library's reading).
 * n_mined / n_correct are ym_tune's arrays (n_gaps x n_taus, row-major),
 * n_truth the number of reference pairs (truth_off[n_pairs]).  F1 =
 * 2 correct / (mined + n_truth) (0 when both are 0), compared exactly in
 * integers; among equal values the first entry in row-major order (the
 * earliest gap, then the earliest threshold) is chosen.  Host only, no device
 * work.  YM_EINVAL for NULL pointers, empty sweeps or counts that are not
 * 0 <= correct <= min(mined, n_truth). */
typedef struct {
  int32_t gap_index, tau_index;
  int64_t n_mined, n_correct;
  double precision, recall, f1;
} ym_tune_choice;
ym_status ym_tune_select(const int64_t *n_mined, const int64_t *n_correct, int32_t n_gaps, int32_t n_taus,
                         int64_t n_truth, ym_tune_choice *out);

/* Bidirectional mining (Section 5: a second classifier trained in the other
 * direction, results joined without duplicates).  Mines the batch forward
 * with (lex_fwd, fwd) and with source and target swapped with (lex_rev, rev),
 * maps the reverse pairs back to (source index, target index), and returns
 * per document pair the union ordered by (source, target) index.  A pair
 * found both ways carries its forward score; align_score is the forward
 * H[n][m]. */
ym_status ym_mine_bidirectional(ym_ctx *ctx, const ym_lexicon *lex_fwd, const ym_lexicon *lex_rev,
                                const ym_batch *batch, const ym_params *fwd, const ym_params *rev, ym_result **out);

/* ------------------------------------------------------------ launch tuning */

/* Launch configuration of a context (applies to every entry point; set it
 * before starting a server on the context).  None of these choices changes a
 * result: they only change how work is split over workgroups. */
typedef struct {
  int32_t sim_kernel;         /* similarity kernel: 1 one lane per target sentence (default); 2 the same,
                                 with the reads of target sentences longer than 32 tokens split over the
                                 lanes a chunk leaves spare; 0 bit-sliced tiles of one wave; 3 and 4
                                 bit-sliced 64-row tiles shared by four waves, target chunks of at most
                                 1,280 (3) or 2,048 (4) tokens */
  int32_t item_rows;          /* source sentences per similarity work item: 64, 128 (default) or 256 */
  int32_t nw_pairs_per_group; /* document pairs per NW workgroup, one wave each: 1 (default), 2 or 4 */
  int32_t nw_large;           /* pairs of 449 or more source sentences, swept with their 64-row strips
                                 pipelined over several waves: 1 (default) the strips of all such pairs
                                 spread over every CU (a persistent grid taking strips in dependency
                                 order); 0 one 16-wave workgroup per pair */
} ym_tuning;

/* Set / read the configuration.  YM_EINVAL for values outside the lists above. */
ym_status ym_set_tuning(ym_ctx *ctx, const ym_tuning *tuning);
ym_status ym_get_tuning(ym_ctx *ctx, ym_tuning *tuning);

/* Autotuner: times the whole path (similarity, NW, compaction) on `sample`
 * with HIP events on the context's stream, `reps` timed passes per candidate
 * after one untimed pass, first over the fifteen (sim_kernel, item_rows) pairs,
 * then over the NW workgroup sizes with the best of them, then (when the
 * sample holds a pair of 449 or more source sentences) both nw_large, compared
 * on the NW kernels' own time (unless kernel timing is enabled on the context
 * or holds events not read yet, which it would consume: then on whole
 * passes).  The fastest
 * configuration is applied to the context and returned in *best, its mean
 * time per pass in *best_ms (may be NULL).  On error the previous
 * configuration is kept. */
ym_status ym_autotune(ym_ctx *ctx, const ym_lexicon *lex, const ym_batch *sample, const ym_params *params,
                      int32_t reps, ym_tuning *best, double *best_ms);

/* Failure injection for tests of the error path: the limit, in ticks of the
 * device's 100 MHz constant clock, of one bounded wait of the pipelined NW
 * sweep (pairs of 448 or more source sentences).  ticks < 0 restores the
 * default (20 s); 0 makes every such wait give up at once, so every pair that
 * needs the pipelined sweep fails with YM_EDEVICE while every kernel still
 * runs to its end. */
ym_status ym_set_wait_limit(ym_ctx *ctx, int64_t ticks);

/* ------------------------------------------------------------ kernel timing */

/* Record HIP events around every kernel the context launches (on the stream
 * the kernel runs on).  Off by default; costs two event records per launch. */
ym_status ym_profile_enable(ym_ctx *ctx, int enable);
/* Summed kernel durations in milliseconds since the last read, by kernel:
 * ms[0] similarity, ms[1] Needleman-Wunsch, ms[2] scan + compaction,
 * ms[3] source-token translation; launches[k] counts the launches.  Waits
 * for the recorded events. */
ym_status ym_profile_read(ym_ctx *ctx, double ms[4], int64_t launches[4]);

/* -------------------------------------------------- serving (continuous batching) */

typedef struct {
  int32_t max_pairs_per_step; /* descriptor-table capacity of one batch step */
  int64_t max_cells_per_step; /* cap on sum n*m admitted into one step */
  int32_t use_graph;          /* capture each step (copy-in, kernels, copy-out) in a hipGraph, updated in place between steps */
} ym_server_opts;

/* Start a serving loop over a resident lexicon and fixed parameters
 * (document pairs are mined independently of each other, Section 4, so
 * pairs that arrive apart can share a batch step).  A
 * background thread admits submitted requests as slots and HBM budget free
 * up, packs them into the next batch step and runs the same kernels as
 * ym_mine; requests that arrive while a step runs join a later step. */
ym_status ym_server_start(ym_ctx *ctx, const ym_lexicon *lex, const ym_params *params,
                          const ym_server_opts *opts, ym_server **out);
/* Submit one document pair (a batch with n_pairs == 1, host memory, copied
 * before return).  YM_EBUDGET if the pair alone exceeds the HBM budget. */
ym_status ym_submit(ym_server *srv, const ym_batch *one_pair, uint64_t *ticket);
/* YM_EPENDING until finished; then the result (caller frees) and the ticket
 * is retired.  timeout_us < 0 waits without limit, 0 polls. */
ym_status ym_poll(ym_server *srv, uint64_t ticket, int64_t timeout_us, ym_result **out);
/* Next finished ticket in completion order (done, failed or cancelled) and
 * its completion time in ns of CLOCK_MONOTONIC.  The ticket still has to be
 * retired with ym_poll.  YM_EPENDING if none finishes within timeout_us
 * (< 0: wait without limit). */
ym_status ym_server_next_done(ym_server *srv, int64_t timeout_us, uint64_t *ticket, int64_t *done_ns);
/* Mark a request cancelled: if not yet admitted it never runs; if running its
 * result is dropped.  ym_poll then returns YM_ECANCELLED. */
ym_status ym_cancel(ym_server *srv, uint64_t ticket);
/* Stop: finishes running steps, cancels what was not admitted, joins. */
ym_status ym_server_stop(ym_server *srv);
/* Counters: steps run, requests completed, cells processed. */
ym_status ym_server_stats(const ym_server *srv, int64_t *steps, int64_t *completed, int64_t *cells);
/* Graph mode (use_graph): executable graphs instantiated and updated in place
 * (hipGraphExecUpdate) so far, over both step slots. */
ym_status ym_server_graph_stats(const ym_server *srv, int64_t *instantiations, int64_t *updates);

#ifdef __cplusplus
}
#endif
#endif /* YMINE_H */
