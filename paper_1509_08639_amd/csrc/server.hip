// Serving loop with continuous batching (ym_server_* in include/ymine.h).
//
// Submitted document pairs wait in a FIFO.  A scheduler thread owns two step
// slots, each with its own stream, pinned staging and device buffers.  When a
// slot is free it admits waiting requests in arrival order while the step
// stays within the pair / cell caps and the HBM budget left over by the other
// slot, packs them into one ragged batch, and enqueues copy-in, the mining
// kernels and copy-out on its stream.  While one step runs on the GPU the next
// one is packed and enqueued on the other stream, so requests that arrive
// during a step are served by the following one and both steps overlap on the
// device.  Each request's result is cut out of its step's output and handed
// to ym_poll; a request's result does not depend on which requests shared its
// step (every pair is computed on its own).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/ymine.h"
#include "ym_internal.h"
#include "ym_runtime.h"

using namespace ym;

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

enum State { kPending = 0, kRunning = 1, kDone = 2, kCancelled = 3, kFailed = 4 };

struct Request {
  uint64_t ticket = 0;
  std::vector<int64_t> ssent, tsent;  // sentence offsets rebased to 0 ([n+1], [m+1])
  std::vector<int32_t> stok, ttok;
  int64_t n = 0, m = 0;
  size_t bytes = 0;  // device bytes this request adds to a step
  int64_t t_submit = 0, t_done = 0;
  int state = kPending;
  bool cancel = false;
  ym_status status = YM_OK;
  std::string error;  // why the request's step failed
  ym_result *result = nullptr;
};

// Device bytes one request adds to a step: its inputs, workspace share and outputs.
size_t request_bytes(int64_t n, int64_t m, int64_t ntok_s, int64_t ntok_t) {
  return a256((size_t)(n + m + 2) * 8) + a256((size_t)(ntok_s + ntok_t) * 4 + 8) + trans_bytes(ntok_s) + pair_bytes(n, m) +
         a256((size_t)std::min(n, m) * 12 + 16) + 1024;
}

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  Staging stage;
  DevBuf dev;      // inputs | workspace | outputs
  HostBuf hin;     // packed inputs
  HostBuf hout;    // outputs copied back
  std::vector<Request *> reqs;
  std::vector<int64_t> sdo, tdo;
  bool busy = false;
  int64_t cap = 0;  // output capacity of the step
  size_t off_out = 0;
  ym_status launch_status = YM_OK;
  // executable graphs of the last steps (graph mode), one per step shape:
  // without and with the large-pair NW launch
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  int64_t graph_updates = 0, graph_instantiations = 0;
};

}  // namespace

struct ym_server {
  ym_ctx *ctx = nullptr;
  int device = 0;
  const ym_lexicon *lex = nullptr;
  ym_params prm{};
  ym_server_opts opts{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> pending;
  std::unordered_map<uint64_t, Request *> all;
  std::deque<std::pair<uint64_t, int64_t>> done_q;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread th;
  Slot slots[2];
  int64_t n_steps = 0, n_completed = 0, n_cells = 0;
};

namespace {

// Pack the slot's requests into one batch and enqueue the step on its stream.
ym_status launch_step(ym_server *S, Slot &sl) {
  const int64_t P = (int64_t)sl.reqs.size();
  sl.sdo.assign(P + 1, 0);
  sl.tdo.assign(P + 1, 0);
  int64_t nts = 0, ntt = 0;
  for (int64_t k = 0; k < P; k++) {
    Request *r = sl.reqs[k];
    sl.sdo[k + 1] = sl.sdo[k] + r->n;
    sl.tdo[k + 1] = sl.tdo[k] + r->m;
    nts += (int64_t)r->stok.size();
    ntt += (int64_t)r->ttok.size();
  }
  const int64_t NS = sl.sdo[P], NT = sl.tdo[P];
  const size_t s1 = a256((size_t)(NS + 1) * 8), s2 = a256((size_t)(NT + 1) * 8), s3 = a256((size_t)nts * 4 + 4),
               s4 = a256((size_t)ntt * 4 + 4);
  const size_t in_bytes = s1 + s2 + s3 + s4;
  Chunk ch;
  ch.layout(sl.sdo.data(), sl.tdo.data(), 0, P, S->ctx->item_rows);
  sl.cap = ch.slots;
  const size_t o1 = a256((size_t)(P + 1) * 8), o2 = a256((size_t)P * 4 + 4), o3 = a256((size_t)sl.cap * 4 + 4);
  const size_t out_bytes = o1 + o2 + 3 * o3;
  ym_status s;
  if ((s = sl.hin.reserve(in_bytes))) return s;
  if ((s = sl.hout.reserve(out_bytes))) return s;
  const size_t head = trans_bytes(nts);
  if ((s = sl.dev.reserve(in_bytes + head + a256(ch.bytes) + out_bytes, true))) return s;

  // pack inputs (global sentence offsets)
  char *h = (char *)sl.hin.ptr;
  int64_t *hs = (int64_t *)h, *ht = (int64_t *)(h + s1);
  int32_t *hst = (int32_t *)(h + s1 + s2), *htt = (int32_t *)(h + s1 + s2 + s3);
  int64_t si = 0, ti = 0, sb = 0, tb = 0;
  hs[0] = 0;
  ht[0] = 0;
  for (int64_t k = 0; k < P; k++) {
    Request *r = sl.reqs[k];
    for (int64_t i = 1; i <= r->n; i++) hs[++si] = sb + r->ssent[i];
    for (int64_t j = 1; j <= r->m; j++) ht[++ti] = tb + r->tsent[j];
    if (!r->stok.empty()) std::memcpy(hst + sb, r->stok.data(), r->stok.size() * 4);
    if (!r->ttok.empty()) std::memcpy(htt + tb, r->ttok.data(), r->ttok.size() * 4);
    sb += (int64_t)r->stok.size();
    tb += (int64_t)r->ttok.size();
  }
  char *d = (char *)sl.dev.ptr;
  // Graph mode: the step's copies and kernels are captured into a graph; the
  // previous step's executable graph is updated in place when the topology
  // matches (hipGraphExecUpdate), else a new one is instantiated.  The slot's
  // events are recorded after the launch, outside the graph.
  const bool graph = S->opts.use_graph != 0;
  sl.stage.caller_syncs = graph;
  hipError_t e;
  if (graph) {
    // the staging buffer is free once the slot's previous step has read it
    if ((e = hipEventSynchronize(sl.stage.done))) return hip_fail(e, "staging wait");
    if ((e = hipStreamBeginCapture(sl.stream, hipStreamCaptureModeRelaxed))) return hip_fail(e, "begin capture");
  }
  auto abort_capture = [&]() {
    if (!graph) return;
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(sl.stream, &g) == hipSuccess && g) hipGraphDestroy(g);
    (void)hipGetLastError();
  };
  e = hipMemcpyAsync(d, h, in_bytes, hipMemcpyHostToDevice, sl.stream);
  if (e) {
    abort_capture();
    return hip_fail(e, "step upload");
  }
  DevBatch b;
  b.src_sent_off = (const int64_t *)d;
  b.tgt_sent_off = (const int64_t *)(d + s1);
  b.src_tok = (const int32_t *)(d + s1 + s2);
  b.tgt_tok = (const int32_t *)(d + s1 + s2 + s3);
  b.n_src_sent = NS;
  b.n_tgt_sent = NT;
  b.n_src_tok = nts;
  b.n_tgt_tok = ntt;
  if ((s = translate_batch(S->ctx, S->lex, b, d + in_bytes, sl.stream))) {
    abort_capture();
    return s;
  }
  char *ws = d + in_bytes + head;
  char *ob = ws + a256(ch.bytes);
  sl.off_out = in_bytes + head + a256(ch.bytes);
  ym_device_out o;
  o.pair_off = (int64_t *)ob;
  o.align_score = (float *)(ob + o1);
  o.src_idx = (int32_t *)(ob + o1 + o2);
  o.tgt_idx = (int32_t *)(ob + o1 + o2 + o3);
  o.score = (float *)(ob + o1 + o2 + 2 * o3);
  o.status = nullptr;  // a failed pair is told by its NaN score (finish_step)
  if ((s = run_chunk(S->ctx, S->lex, b, &S->prm, sl.sdo.data(), sl.tdo.data(), ch, ws, o, sl.stream, nullptr,
                     &sl.stage))) {
    abort_capture();
    return s;
  }
  e = hipMemcpyAsync(sl.hout.ptr, ob, out_bytes, hipMemcpyDeviceToHost, sl.stream);
  if (e) {
    abort_capture();
    return hip_fail(e, "step download");
  }
  if (graph) {
    hipGraph_t g = nullptr;
    if ((e = hipStreamEndCapture(sl.stream, &g)) || !g) return hip_fail(e ? e : hipErrorUnknown, "end capture");
    bool updated = false;
    hipGraphExec_t &ex = sl.exec[ch.n_big > 0 ? 1 : 0];
    if (ex) {
      hipGraphNode_t err_node = nullptr;
      hipGraphExecUpdateResult res = hipGraphExecUpdateError;
      if (hipGraphExecUpdate(ex, g, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess) {
        updated = true;
        sl.graph_updates++;
      } else {
        (void)hipGetLastError();
        hipGraphExecDestroy(ex);
        ex = nullptr;
      }
    }
    if (!updated) {
      if ((e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0))) {
        hipGraphDestroy(g);
        ex = nullptr;
        return hip_fail(e, "graph instantiate");
      }
      sl.graph_instantiations++;
    }
    hipGraphDestroy(g);
    if ((e = hipGraphLaunch(ex, sl.stream))) return hip_fail(e, "graph launch");
    if ((e = hipEventRecord(sl.stage.done, sl.stream))) return hip_fail(e, "staging event");
  }
  if ((e = hipEventRecord(sl.done, sl.stream))) return hip_fail(e, "step event");
  return YM_OK;
}

// Cut the step's outputs into per-request results.
void finish_step(ym_server *S, Slot &sl, ym_status st) {
  const int64_t P = (int64_t)sl.reqs.size();
  const char *h = (const char *)sl.hout.ptr;
  const size_t o1 = a256((size_t)(P + 1) * 8), o2 = a256((size_t)P * 4 + 4), o3 = a256((size_t)sl.cap * 4 + 4);
  const int64_t *po = (const int64_t *)h;
  const float *al = (const float *)(h + o1);
  const int32_t *src = (const int32_t *)(h + o1 + o2);
  const int32_t *tgt = (const int32_t *)(h + o1 + o2 + o3);
  const float *sc = (const float *)(h + o1 + o2 + 2 * o3);
  const int64_t t = now_ns();
  int64_t cells = 0;
  for (int64_t k = 0; k < P; k++) {
    Request *r = sl.reqs[k];
    cells += r->n * r->m;
    r->t_done = t;
    if (st != YM_OK) {
      r->state = kFailed;
      r->status = st;
    } else if (r->cancel) {
      r->state = kCancelled;
    } else if (std::isnan(al[k])) {  // the pair's pipelined sweep gave up on a bounded wait
      r->state = kFailed;
      r->status = YM_EDEVICE;
      r->error = "the pipelined Needleman-Wunsch sweep gave up on a bounded wait";
    } else {
      const int64_t a = po[k], c = po[k + 1] - po[k];
      ym_result *res = (ym_result *)calloc(1, sizeof(ym_result));
      if (res) {
        res->n_pairs = 1;
        res->n_out = c;
        res->pair_off = (int64_t *)malloc(16);
        res->align_score = (float *)malloc(4);
        res->src_idx = (int32_t *)malloc((size_t)std::max<int64_t>(c, 1) * 4);
        res->tgt_idx = (int32_t *)malloc((size_t)std::max<int64_t>(c, 1) * 4);
        res->score = (float *)malloc((size_t)std::max<int64_t>(c, 1) * 4);
      }
      if (!res || !res->pair_off || !res->align_score || !res->src_idx || !res->tgt_idx || !res->score) {
        ym_result_free(res);
        r->state = kFailed;
        r->status = YM_ENOMEM;
      } else {
        res->pair_off[0] = 0;
        res->pair_off[1] = c;
        res->align_score[0] = al[k];
        if (c) {
          std::memcpy(res->src_idx, src + a, (size_t)c * 4);
          std::memcpy(res->tgt_idx, tgt + a, (size_t)c * 4);
          std::memcpy(res->score, sc + a, (size_t)c * 4);
        }
        r->result = res;
        r->state = kDone;
      }
    }
    S->done_q.push_back({r->ticket, r->t_done});
    if (S->done_q.size() > ((size_t)1 << 20)) S->done_q.pop_front();
  }
  S->n_steps++;
  S->n_completed += P;
  S->n_cells += cells;
  sl.reqs.clear();
  sl.busy = false;
}

void scheduler(ym_server *S) {
  hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    // retire finished steps
    bool progressed = false;
    for (Slot &sl : S->slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipSuccess) {
        finish_step(S, sl, YM_OK);
        progressed = true;
      } else if (q != hipErrorNotReady) {
        finish_step(S, sl, hip_fail(q, "step"));
        progressed = true;
      }
    }
    if (progressed) S->cv_done.notify_all();
    bool busy_any = S->slots[0].busy || S->slots[1].busy;
    if (S->stop && !busy_any) break;
    // admit into a free slot
    if (!S->stop && !S->pending.empty()) {
      Slot *free_slot = !S->slots[0].busy ? &S->slots[0] : (!S->slots[1].busy ? &S->slots[1] : nullptr);
      if (free_slot) {
        Slot &other = free_slot == &S->slots[0] ? S->slots[1] : S->slots[0];
        const size_t other_bytes = other.dev.cap;  // device bytes held by the other slot
        const size_t budget = S->ctx->budget > other_bytes ? S->ctx->budget - other_bytes : 0;
        size_t bytes = 0;
        int64_t cells = 0;
        while (!S->pending.empty() && (int64_t)free_slot->reqs.size() < S->opts.max_pairs_per_step) {
          Request *r = S->pending.front();
          if (r->cancel) {
            S->pending.pop_front();
            r->state = kCancelled;
            r->t_done = now_ns();
            S->done_q.push_back({r->ticket, r->t_done});
            S->cv_done.notify_all();
            continue;
          }
          const int64_t c = r->n * r->m;
          if (!free_slot->reqs.empty() && (bytes + r->bytes > budget || cells + c > S->opts.max_cells_per_step)) break;
          if (free_slot->reqs.empty() && r->bytes > budget) break;  // wait for the other slot to drain
          S->pending.pop_front();
          r->state = kRunning;
          free_slot->reqs.push_back(r);
          bytes += r->bytes;
          cells += c;
        }
        if (!free_slot->reqs.empty()) {
          free_slot->busy = true;
          lk.unlock();
          const ym_status st = launch_step(S, *free_slot);
          const std::string why = st != YM_OK ? std::string(ym_last_error()) : std::string();
          lk.lock();
          if (st != YM_OK) {
            hipStreamSynchronize(free_slot->stream);
            for (Request *r : free_slot->reqs) r->error = why;
            finish_step(S, *free_slot, st);
            S->cv_done.notify_all();
          }
          continue;
        }
      }
    }
    busy_any = S->slots[0].busy || S->slots[1].busy;
    if (busy_any) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else if (!S->stop) {
      S->cv_work.wait_for(lk, std::chrono::milliseconds(5));
    }
  }
  // cancel what was never admitted
  while (!S->pending.empty()) {
    Request *r = S->pending.front();
    S->pending.pop_front();
    r->state = kCancelled;
    S->done_q.push_back({r->ticket, now_ns()});
  }
  S->cv_done.notify_all();
}

void free_request(Request *r) {
  if (!r) return;
  ym_result_free(r->result);
  delete r;
}

}  // namespace

extern "C" {

ym_status ym_server_start(ym_ctx *c, const ym_lexicon *L, const ym_params *p, const ym_server_opts *opts,
                          ym_server **out) {
  if (!out) return fail(YM_EINVAL, "NULL out");
  *out = nullptr;
  if (!c || !L) return fail(YM_EINVAL, "NULL context or lexicon");
  ym_status s;
  if ((s = check_params(p))) return s;
  ym_server *S = new (std::nothrow) ym_server();
  if (!S) return fail(YM_ENOMEM, "server allocation");
  S->ctx = c;
  S->device = c->device;
  S->lex = L;
  S->prm = *p;
  S->opts.max_pairs_per_step = opts && opts->max_pairs_per_step > 0 ? opts->max_pairs_per_step : 256;
  S->opts.max_cells_per_step = opts && opts->max_cells_per_step > 0 ? opts->max_cells_per_step : ((int64_t)1 << 26);
  S->opts.use_graph = opts ? opts->use_graph : 0;
  hipSetDevice(c->device);
  hipError_t e = hipSuccess;
  for (Slot &sl : S->slots) {
    if (!e) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (!e) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (!e) e = hipEventCreateWithFlags(&sl.stage.done, hipEventDisableTiming);
  }
  if (!e) {
    std::lock_guard<std::mutex> lk(c->mu);
    if ((s = ensure_table(c, p, c->stream)) == YM_OK) e = hipStreamSynchronize(c->stream);
  }
  if (e || s) {
    for (Slot &sl : S->slots) {
      if (sl.stream) hipStreamDestroy(sl.stream);
      if (sl.done) hipEventDestroy(sl.done);
      if (sl.stage.done) hipEventDestroy(sl.stage.done);
    }
    delete S;
    return e ? hip_fail(e, "server start") : s;
  }
  try {
    S->th = std::thread(scheduler, S);
  } catch (...) {
    delete S;
    return fail(YM_ENOMEM, "server thread");
  }
  *out = S;
  return YM_OK;
}

ym_status ym_submit(ym_server *S, const ym_batch *b, uint64_t *ticket) {
  if (!S || !b || !ticket) return fail(YM_EINVAL, "NULL argument");
  if (b->n_pairs != 1) return fail(YM_EINVAL, "ym_submit takes exactly one document pair");
  ym_status s;
  if ((s = check_doc_off(b->src_doc_off, 1, "src_doc_off")) || (s = check_doc_off(b->tgt_doc_off, 1, "tgt_doc_off")))
    return s;
  const int64_t n = b->src_doc_off[1], m = b->tgt_doc_off[1];
  if ((s = check_pair_shape(n, m, 0))) return s;
  if (!b->src_sent_off || !b->tgt_sent_off) return fail(YM_EINVAL, "NULL sentence offsets");
  if (b->src_sent_off[0] != 0 || b->tgt_sent_off[0] != 0) return fail(YM_EINVAL, "sentence offsets must start at 0");
  for (int64_t i = 0; i < n; i++) {
    if (b->src_sent_off[i + 1] < b->src_sent_off[i]) return fail(YM_EINVAL, "src_sent_off decreases");
    if (b->src_sent_off[i + 1] - b->src_sent_off[i] > kMaxSentTokens)
      return fail(YM_EINVAL, "source sentence %lld has more than %d tokens", (long long)i, kMaxSentTokens);
  }
  for (int64_t j = 0; j < m; j++) {
    if (b->tgt_sent_off[j + 1] < b->tgt_sent_off[j]) return fail(YM_EINVAL, "tgt_sent_off decreases");
    if (b->tgt_sent_off[j + 1] - b->tgt_sent_off[j] > kMaxSentTokens)
      return fail(YM_EINVAL, "target sentence %lld has more than %d tokens", (long long)j, kMaxSentTokens);
  }
  const int64_t ns = b->src_sent_off[n], nt = b->tgt_sent_off[m];
  if ((ns && !b->src_tok) || (nt && !b->tgt_tok)) return fail(YM_EINVAL, "NULL tokens");
  const size_t bytes = request_bytes(n, m, ns, nt);
  if (bytes > S->ctx->budget)
    return fail(YM_EBUDGET, "request needs %zu device bytes, budget is %zu", bytes, S->ctx->budget);
  Request *r = new (std::nothrow) Request();
  if (!r) return fail(YM_ENOMEM, "request allocation");
  try {
    r->ssent.assign(b->src_sent_off, b->src_sent_off + n + 1);
    r->tsent.assign(b->tgt_sent_off, b->tgt_sent_off + m + 1);
    r->stok.assign(b->src_tok, b->src_tok + ns);
    r->ttok.assign(b->tgt_tok, b->tgt_tok + nt);
  } catch (...) {
    delete r;
    return fail(YM_ENOMEM, "request copy");
  }
  r->n = n;
  r->m = m;
  r->bytes = bytes;
  r->t_submit = now_ns();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
      delete r;
      return fail(YM_ECANCELLED, "server is stopping");
    }
    r->ticket = S->next_ticket++;
    S->all[r->ticket] = r;
    S->pending.push_back(r);
    *ticket = r->ticket;
  }
  S->cv_work.notify_one();
  return YM_OK;
}

ym_status ym_poll(ym_server *S, uint64_t ticket, int64_t timeout_us, ym_result **out) {
  if (!S || !out) return fail(YM_EINVAL, "NULL argument");
  *out = nullptr;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return fail(YM_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  Request *r = it->second;
  auto finished = [&] { return r->state >= kDone; };
  if (!finished()) {
    if (timeout_us == 0) return YM_EPENDING;
    if (timeout_us < 0)
      S->cv_done.wait(lk, finished);
    else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), finished))
      return YM_EPENDING;
  }
  S->all.erase(it);
  const int st = r->state;
  const ym_status code = r->status;
  const std::string why = r->error;
  if (st == kDone) {
    *out = r->result;
    r->result = nullptr;
  }
  free_request(r);
  if (st == kCancelled) return fail(YM_ECANCELLED, "request %llu was cancelled", (unsigned long long)ticket);
  if (st == kFailed) return fail(code, "request %llu failed: %s", (unsigned long long)ticket, why.c_str());
  return YM_OK;
}

ym_status ym_server_next_done(ym_server *S, int64_t timeout_us, uint64_t *ticket, int64_t *done_ns) {
  if (!S || !ticket) return fail(YM_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(S->mu);
  auto ready = [&] { return !S->done_q.empty(); };
  if (!ready()) {
    if (timeout_us == 0) return YM_EPENDING;
    if (timeout_us < 0)
      S->cv_done.wait(lk, [&] { return ready() || (S->stop && S->all.empty()); });
    else
      S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
    if (!ready()) return YM_EPENDING;
  }
  *ticket = S->done_q.front().first;
  if (done_ns) *done_ns = S->done_q.front().second;
  S->done_q.pop_front();
  return YM_OK;
}

ym_status ym_cancel(ym_server *S, uint64_t ticket) {
  if (!S) return fail(YM_EINVAL, "NULL server");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return fail(YM_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  it->second->cancel = true;
  return YM_OK;
}

ym_status ym_server_stop(ym_server *S) {
  if (!S) return fail(YM_EINVAL, "NULL server");
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->th.joinable()) S->th.join();
  hipSetDevice(S->device);
  for (Slot &sl : S->slots) {
    hipStreamSynchronize(sl.stream);
    sl.dev.release();
    sl.hin.release();
    sl.hout.release();
    sl.stage.buf.release();
    for (hipGraphExec_t &x : sl.exec)
      if (x) hipGraphExecDestroy(x);
    hipEventDestroy(sl.done);
    hipEventDestroy(sl.stage.done);
    hipStreamDestroy(sl.stream);
  }
  for (auto &kv : S->all) free_request(kv.second);
  delete S;
  return YM_OK;
}

ym_status ym_server_stats(const ym_server *S, int64_t *steps, int64_t *completed, int64_t *cells) {
  if (!S) return fail(YM_EINVAL, "NULL server");
  ym_server *T = const_cast<ym_server *>(S);
  std::lock_guard<std::mutex> lk(T->mu);
  if (steps) *steps = S->n_steps;
  if (completed) *completed = S->n_completed;
  if (cells) *cells = S->n_cells;
  return YM_OK;
}

ym_status ym_server_graph_stats(const ym_server *S, int64_t *instantiations, int64_t *updates) {
  if (!S) return fail(YM_EINVAL, "NULL server");
  ym_server *T = const_cast<ym_server *>(S);
  std::lock_guard<std::mutex> lk(T->mu);
  int64_t a = 0, u = 0;
  for (const Slot &sl : S->slots) {
    a += sl.graph_instantiations;
    u += sl.graph_updates;
  }
  if (instantiations) *instantiations = a;
  if (updates) *updates = u;
  return YM_OK;
}

}  // extern "C"
