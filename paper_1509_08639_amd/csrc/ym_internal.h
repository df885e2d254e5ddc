// Internal definitions shared by the kernels and the host runtime of libymine.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ym {

constexpr int32_t kEmpty = -1;          // empty hash slot key (lexicon ids are >= 0)
constexpr uint32_t kHitBit = 0x80000000u;  // "target id is in X_i" flag of a mask word
constexpr int kPosBits = 31;            // source positions per two-row step (bit 31: hit bit)

// Similarity kernel tiling.
constexpr int kSimThreads = 256;        // 4 waves; each wave owns one source sentence at a time
constexpr int kSimWaves = kSimThreads / 64;
constexpr int kTcap = 1024;             // max target tokens staged per chunk (and per sentence)
constexpr int kUcap = 2 * kTcap;        // LDS hash slots for the chunk's distinct target ids
constexpr int kLogUcap = 11;
constexpr int kJcap = 64;               // max target sentences per chunk (one per lane)
constexpr int kTdocCap = kTcap + 3 * kJcap;  // staged ids, each sentence padded to a multiple of 4
static_assert(kJcap <= kSimThreads && kJcap == 64, "one lane per target sentence of a chunk");
constexpr int kItemRows = 128;          // source sentences per work item (two 64-row strips)
constexpr int kMinItemRows = 64, kMaxItemRows = 256;  // range of the tunable rows per similarity item
constexpr int kMaxSentTokens = 1024;    // longest sentence the host entry points accept
// Most sentences per document: one 64-row strip of a pair's scores, which the
// NW sweep reads through one buffer resource, then stays below 2 GiB.
constexpr int64_t kMaxDocSents = 1 << 22;
constexpr int kTabLen = 64;             // score table covers sentence lengths < 64
constexpr int kLogTabLen = 6;

// NW kernel staging.
constexpr int kDirLds = 1856;           // direction words held in LDS (covers 168 x 160; 9.25 KB with the row, four waves per SIMD)
constexpr int kRowLds = 512;            // boundary-row floats held in LDS

static_assert((1 << kLogUcap) == kUcap, "hash capacity");

// NW direction words per DP row: codes are packed 16 per word by sweep step,
// and a row's m cells span at most ceil(m/16) + 1 words.
__host__ __device__ constexpr int64_t nw_dir_row_words(int64_t m) { return (m + 15) / 16 + 1; }

// Pairs of at least kNwBigStrips strips of 64 rows ("large pairs") are swept
// with their strips pipelined over several waves: either the waves of one
// kNwBigWaves-wave workgroup per pair, or every wave of a persistent grid
// (strips taken in dependency order); smaller pairs by one wave each.
constexpr int kNwBigStrips = 8, kNwBigWaves = 16;
__host__ __device__ constexpr bool nw_is_big(int64_t n) { return (n + 63) / 64 >= kNwBigStrips; }
// Persistent-grid sweep of the large pairs: workgroups of four independent
// waves, at most kNwSplitGroupsPerCu per CU of a 256-CU device.
constexpr int kNwSplitWaves = 4, kNwSplitGroupsPerCu = 2, kNwSplitCus = 256;
// Its control words per gap penalty: a ticket counter and the launch's tag,
// then per large pair {strips finished, give-up flag, H[n][m] and its tag as
// one 8-byte entry} (an even count, so every entry stays 8-byte aligned).
constexpr int kNwCtrlHead = 2, kNwCtrlPerPair = 4;

// Score layout of one n x m block: rows in strips of 64 (the last one has
// R = n - 64 (strips - 1) rows); inside a strip, anti-diagonal t = l + c is a
// row of R slots and cell (l, c) sits at t * R + l.  A strip holds
// (m + R - 1) * R slots, of which R * m are cells; the NW sweep reads one
// anti-diagonal per step as one contiguous run.
__host__ __device__ constexpr int64_t score_slots(int64_t n, int64_t m) {
  return (n <= 0 || m <= 0) ? 0
                            : ((n - 1) / 64) * (m + 63) * 64 + (m + (n - 64 * ((n - 1) / 64)) - 1) * (n - 64 * ((n - 1) / 64));
}
// a pair's block in a chunk, rounded up to 16 bytes (blocks start 16-byte aligned)
__host__ __device__ constexpr int64_t score_block(int64_t n, int64_t m) { return (score_slots(n, m) + 3) & ~int64_t(3); }
// The similarity kernels address a pair's scores with 32-bit offsets from the
// start of its block, so a pair's block must stay below 2^31 slots (n = m =
// 46,000 is about the largest square pair); the host rejects larger pairs.
constexpr int64_t kMaxPairSlots = ((int64_t)1 << 31) - 4;
// offset of score (i, c) inside its pair's block (layout: score_slots)
__host__ __device__ inline int64_t score_pos(int i, int c, int n, int m) {
  const int s = i >> 6, l = i & 63;
  const int R = (n - (s << 6)) < 64 ? (n - (s << 6)) : 64;
  return (int64_t)s * (m + 63) * 64 + (int64_t)(l + c) * R + l;
}

// One document pair of a chunk.
struct PairDesc {
  int64_t src_sent0;  // global index of its first source sentence
  int64_t tgt_sent0;  // global index of its first target sentence
  int64_t s_off;      // offset of its n x m score block (floats)
  int64_t out_off;    // offset of its min(n, m) output slots
  int64_t dir_off;    // offset of its direction words in global scratch (-1: LDS)
  int64_t row_off;    // offset of its boundary row in global scratch (-1: LDS)
  int64_t rm_off;     // offset of its n x m block in row-major debug buffers
  int32_t n, m;
};

// Similarity work item: source sentences [i0, i1) of pair `pair` against all
// its target sentences.
struct SimItem {
  int32_t pair;
  int32_t i0, i1;
  int32_t n, m;  // the pair's fields the similarity kernel reads, copied so
  int32_t pad;   // that an item is one load (no dependent descriptor load)
  int64_t src_sent0, tgt_sent0, s_off, rm_off;
};

// Lexicon as resident in HBM: open-addressing table of {key, count, offset, 0}
// slots (linear probing, load <= 1/2) over a CSR value array.
struct LexDev {
  const int4 *slots;  // two int4 per slot: {key, count, offset, -1}, translation record
  const int32_t *vals;
  uint32_t mask;
  int32_t shift;
  const int4 *dense;  // translation record of every id below dense_n (nullptr: none)
  int32_t dense_n;
};

// Lexicons whose keys are all below this get a dense record table too (16
// bytes per id, 256 MB at most): the translation pass then reads a token's
// record directly instead of probing the hash table.
constexpr int32_t kDenseKeys = 1 << 24;

struct SimArgs {
  const SimItem *items;
  int64_t n_items;
  const PairDesc *descs;
  const int64_t *src_sent_off;
  const int32_t *src_tok;
  const int64_t *tgt_sent_off;
  const int32_t *tgt_tok;
  int64_t n_src_sent, n_tgt_sent, n_src_tok, n_tgt_tok;
  LexDev lex;
  const int4 *trans;  // translations of every source token (translate_kernel)
  float w0, w1, w2, w3;
  const float *table;  // kTabLen^4 scores for short sentences
  float *S;
  int32_t *ms_out;  // optional
  int32_t *mt_out;  // optional
};

struct NwArgs {
  const PairDesc *descs;
  int64_t n_pairs;
  const float *S;
  float gap, tau;
  uint32_t *dir_scratch;
  float *row_scratch;
  int32_t *slot_src, *slot_tgt;
  float *slot_score;
  int32_t *counts;      // [n_pairs] accepted pairs
  float *align;         // [n_pairs] H[n][m] (global pair index = pair_base + local)
  int64_t pair_base;
  const int32_t *big;   // [n_big] local indices of the large pairs (nw_is_big)
  const int32_t *order; // [n_pairs] local pair indices, largest first (launch order of the one-wave sweeps)
  int64_t n_big;
  char *moves;          // optional: forward paths
  const int64_t *moves_off;  // [n_pairs] (local) offsets into moves
  int32_t *n_moves;     // optional [n_pairs] (global index)
  uint64_t wait_ticks;  // limit of one bounded wait of the pipelined sweep (0: give up at once)
  int32_t *status;      // optional: set to kStatusWaitGaveUp when a pair's sweep gives up
  // Several gap penalties in one launch (grid y = gap index g): gaps[g]
  // replaces `gap`, and the outputs and scratch of gap g lie g strides (in
  // elements) after those above.  gaps == nullptr: one gap, `gap`.
  const float *gaps = nullptr;
  int32_t n_gaps = 1;
  int64_t g_dirs = 0, g_rows = 0, g_slots = 0, g_counts = 0, g_align = 0;
  // Large pairs swept by the persistent grid (split = 1) instead of one
  // workgroup each: big_strip0[k] is the first ticket of large pair k (its
  // strips take consecutive tickets; big_strip0[n_big] is the total), ctrl
  // the control words (kNwCtrlHead + kNwCtrlPerPair * n_big per gap, g_ctrl
  // apart), and boundary rows hold {H, tag} entries of 8 bytes.
  int32_t split = 0;
  const int32_t *big_strip0 = nullptr;
  const int32_t *ticket_big = nullptr;  // [n_big_strips] large pair (index into big) of each ticket
  int64_t n_big_strips = 0;
  int32_t *ctrl = nullptr;
  int64_t g_ctrl = 0;
};

// Device status word of a call: 0, or the code of the first device failure.
constexpr int32_t kStatusWaitGaveUp = -3;  // equals YM_EDEVICE
// Default limit of one bounded wait (ticks of the 100 MHz constant counter):
// far above any legitimate wait, which is at most one strip sweep.
constexpr uint64_t kNwWaitTicks = 2000000000ull;  // 20 s

// Launch wrappers (kernels.hip).
hipError_t launch_lex_dense(const int32_t *keys, const int32_t *cnts, const int64_t *offs, const int32_t *vals, int64_t n,
                            int4 *dense, hipStream_t st);
hipError_t launch_lex_insert(const int32_t *keys, const int32_t *cnts, const int64_t *offs, const int32_t *vals,
                             int64_t n, int4 *slots, uint32_t mask, int shift, hipStream_t st);
hipError_t launch_translate(const int32_t *tok, int64_t n, const LexDev &L, int4 *out, hipStream_t st);
hipError_t launch_score_table(float w0, float w1, float w2, float w3, float *table, hipStream_t st);
// variant 0: bit-sliced tile kernel; 1: lane-per-target-sentence kernel
hipError_t launch_similarity(const SimArgs &a, int grid, int variant, hipStream_t st);
hipError_t launch_nw(const NwArgs &a, int pairs_per_group, hipStream_t st);
hipError_t launch_scan(const int32_t *counts, int64_t n, int64_t *pair_off_at_p0, int first, hipStream_t st);
hipError_t launch_compact(const PairDesc *descs, int64_t n_pairs, const int32_t *counts, const int64_t *pair_off_at_p0,
                          const int32_t *slot_src, const int32_t *slot_tgt, const float *slot_score, int32_t *out_src,
                          int32_t *out_tgt, float *out_score, hipStream_t st);
hipError_t launch_relayout(const PairDesc *descs, int64_t n_pairs, const float *src, float *dst, int to_diag,
                           hipStream_t st);
hipError_t launch_tune_count(const PairDesc *descs, int64_t n_pairs, int64_t pair_base, const int32_t *counts,
                             const int32_t *ssrc, const int32_t *stgt, const float *sscore, const int64_t *truth_off,
                             const int32_t *truth_src, const int32_t *truth_tgt, const float *taus, int n_taus,
                             unsigned long long *n_mined, unsigned long long *n_correct, hipStream_t st);
hipError_t launch_merge_bi(int64_t n_pairs, const int64_t *po_f, const int32_t *sf, const int32_t *tf, const float *scf,
                           const int64_t *po_r, const int32_t *sr, const int32_t *tr, const float *scr, int32_t *counts,
                           const int64_t *po_out, int32_t *osrc, int32_t *otgt, float *osc, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st);

}  // namespace ym
