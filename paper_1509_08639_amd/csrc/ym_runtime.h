// Host-side runtime structures of libymine (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <utility>
#include <vector>

#include "../../include/ymine.h"
#include "ym_internal.h"

namespace ym {

struct DevBuf {
  void *ptr = nullptr;
  size_t cap = 0;
  ym_status reserve(size_t bytes, bool exact = false);
  void release();
};

struct HostBuf {  // pinned
  void *ptr = nullptr;
  size_t cap = 0;
  ym_status reserve(size_t bytes);
  void release();
};

// Device view of a batch (all pointers on the device).
struct DevBatch {
  const int64_t *src_sent_off, *tgt_sent_off;
  const int32_t *src_tok, *tgt_tok;
  int64_t n_src_sent, n_tgt_sent, n_src_tok, n_tgt_tok;
  const int4 *trans;  // translations of every source token (workspace head)
};

// Workspace head that holds the source-token translations of a batch.
inline size_t trans_bytes(int64_t n_src_tok) { return ((size_t)(n_src_tok > 0 ? n_src_tok : 0) * 16 + 255) & ~size_t(255); }

// Optional debug outputs of a chunk run.
struct DebugOut {
  float *S_rowmajor_out = nullptr;       // if set: the chunk's scores, row-major, go here (device)
  const float *S_rowmajor_in = nullptr;  // if set: use these row-major scores, skip the similarity kernel
  bool sim_only = false;                 // stop after the similarity kernel
  bool reuse_S = false;                  // the workspace already holds this chunk's scores
  int32_t *ms = nullptr, *mt = nullptr;
  char *moves_dev = nullptr; // device buffer for paths
  int64_t moves_base = 0;    // offset of this chunk's first pair in moves_dev
  int32_t *n_moves_dev = nullptr;
  // a gap sweep: the NW kernel runs once for the chunk's n_gaps penalties
  // gaps[0 .. n_gaps) (device), H[n][m] of gap g at align + g * align_stride,
  // and the call stops after it
  const float *gaps = nullptr;
  int64_t align_stride = 0;
};

// Workspace layout of one chunk of pairs [p0, p1).
struct Chunk {
  int64_t p0 = 0, p1 = 0, np = 0, n_items = 0, cells = 0, s_slots = 0, dir_words = 0, row_floats = 0, slots = 0,
          n_big = 0, n_big_strips = 0;
  size_t off_descs = 0, off_items = 0, off_S = 0, off_dirs = 0, off_rows = 0, off_ssrc = 0, off_stgt = 0,
         off_sscore = 0, off_counts = 0, off_moves_off = 0, off_big = 0, off_order = 0, off_strip0 = 0,
         off_tickets = 0, off_ctrl = 0, bytes = 0, host_bytes = 0;
  int item_rows = kItemRows;  // source sentences per similarity work item
  int n_gaps = 1;             // copies of the NW regions (gap penalties swept by one NW launch)
  ym_status layout(const int64_t *sdo, const int64_t *tdo, int64_t p0, int64_t p1, int item_rows, int n_gaps = 1);
  void fill_host(const int64_t *sdo, const int64_t *tdo, char *host) const;
};

ym_status fail(ym_status code, const char *fmt, ...);
ym_status hip_fail(hipError_t e, const char *what);
// Workspace bytes of one pair, with the NW outputs and scratch once per gap penalty of a launch.
size_t pair_bytes(int64_t n, int64_t m, int n_gaps = 1);
// Workspace bytes of a chunk beyond the pair_bytes of its pairs: the
// alignment padding of its regions (fewer than 16) and the fixed part of the
// NW control words.
inline size_t chunk_fixed_bytes(int n_gaps = 1) {
  return 16 * 256 + (size_t)(n_gaps > 1 ? n_gaps : 1) * 4 * kNwCtrlHead + 4;
}
LexDev lex_dev(const ym_lexicon *L);
ym_status check_params(const ym_params *p);
ym_status check_doc_off(const int64_t *o, int64_t n_pairs, const char *what);
// The sizes one document pair may have: at most kMaxDocSents sentences per
// side and fewer than 2^31 score slots (32-bit offsets inside a pair's block).
ym_status check_pair_shape(int64_t n, int64_t m, int64_t pair);
ym_status ensure_table(ym_ctx *c, const ym_params *p, hipStream_t st);
// Resolve the batch's source tokens into `head` (trans_bytes(n_src_tok) bytes) and point b.trans at it.
ym_status translate_batch(ym_ctx *c, const ym_lexicon *L, DevBatch &b, char *head, hipStream_t st);
ym_status plan_chunks(const int64_t *sdo, const int64_t *tdo, int64_t n_pairs, size_t ws_bytes,
                      std::vector<std::pair<int64_t, int64_t>> &chunks, size_t plan_cap = 0, int n_gaps = 1);
// Pinned staging buffer for plan uploads and the event that marks its last
// upload as done (the buffer is rewritten only after that event).
struct Staging {
  HostBuf buf;
  hipEvent_t done = nullptr;
  bool caller_syncs = false;  // the caller waits for and records `done` (work captured into a graph)
};

// Upload a chunk's plan (descriptors, items, ...) into the workspace: on `st`,
// or with `side` on the context's upload stream after the work already on
// `st`, recording c->ev_up when done (the caller makes `st` wait for it).
ym_status upload_plan(ym_ctx *c, const int64_t *sdo, const int64_t *tdo, const Chunk &ch, char *ws, hipStream_t st,
                      Staging *stg, bool side);
// ym_mine_device with the context lock held; `plan_cap` (0: none) bounds each
// chunk's plan so that its upload fits the pinned staging buffer as it is.
ym_status mine_device(ym_ctx *c, const ym_lexicon *L, const ym_device_batch *b, const ym_params *prm, void *workspace,
                      size_t workspace_bytes, const ym_device_out *out, void *stream, size_t plan_cap);
// Pinned staging reserved by ym_create for plan uploads (never grown by the
// allocation-free entry point).
constexpr size_t kStagingBytes = (size_t)8 << 20;
// The allocation-free entry point's device scratch: look up (once per device,
// with that device current) where this device's copy of the static array lives.
ym_status static_scratch_init(int device);

// Enqueue one chunk: its plan upload (unless `plan_ready`), then the kernels.
ym_status run_chunk(ym_ctx *c, const ym_lexicon *L, const DevBatch &b, const ym_params *prm, const int64_t *sdo,
                    const int64_t *tdo, const Chunk &ch, char *ws, const ym_device_out &out, hipStream_t st,
                    const DebugOut *dbg, Staging *stg = nullptr, bool plan_ready = false);

}  // namespace ym

struct ym_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t up_stream = nullptr;  // plan uploads that overlap the translation kernel
  hipEvent_t ev_ws_free = nullptr, ev_up = nullptr;
  ym::Staging stage;
  size_t budget = 0;       // serving HBM budget
  size_t arena_limit = 0;  // workspace cap for host-API calls
  std::mutex mu;           // one host-API call at a time per context
  ym::DevBuf table, in, ws, outb;
  ym::HostBuf host_out;
  float table_w[4] = {0, 0, 0, 0};
  bool table_valid = false;
  // launch configuration (ym_set_tuning / ym_autotune; read when work is enqueued)
  int sim_variant = 1;  // similarity kernel: 1 lane per target sentence (default), 2 the same with reads of long
                        // sentences split over spare lanes (YM_SIM_KERNEL=split), 0 bit-sliced tiles (=tile),
                        // 3 / 4 bit-sliced tiles of four waves, 1,280- / 2,048-token chunks (=bits / =bits2k)
  int item_rows = ym::kItemRows;  // source sentences per similarity work item
  int nw_pairs_per_group = 1;     // NW workgroup size in pairs (one wave each)
  int nw_large = 1;               // large pairs: 1 strips over the whole GPU, 0 one workgroup per pair
  uint64_t nw_wait_ticks = ym::kNwWaitTicks;  // limit of one bounded wait of the pipelined sweep
  // kernel timing
  bool prof = false;
  std::mutex prof_mu;
  std::vector<hipEvent_t> ev_free;
  struct Timed {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Timed> ev_pending;
  hipEvent_t ev_get() {
    if (!ev_free.empty()) {
      hipEvent_t e = ev_free.back();
      ev_free.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

namespace ym {
// Brackets one kernel launch with events when timing is on.
struct KernelTimer {
  ym_ctx *c;
  int kind;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  KernelTimer(ym_ctx *c_, int kind_, hipStream_t st_) : c(c_), kind(kind_), st(st_) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (c && c->prof && hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
      std::lock_guard<std::mutex> lk(c->prof_mu);
      a = c->ev_get();
      b = c->ev_get();
      if (a && b) hipEventRecord(a, st);
    }
  }
  ~KernelTimer() {
    if (a && b) {
      hipEventRecord(b, st);
      std::lock_guard<std::mutex> lk(c->prof_mu);
      c->ev_pending.push_back({kind, a, b});
    }
  }
};
}  // namespace ym
