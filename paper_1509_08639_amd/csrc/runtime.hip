// Host runtime and C ABI of libymine (declared in include/ymine.h).
//
// Contexts own a HIP stream and a device arena; lexicons are normalised on the
// host (sort, merge duplicate keys, deduplicate targets) and inserted into an
// HBM hash table by a kernel.  A batch is planned on the host from its pair
// table (per-pair offsets of the score block, output slots and, for pairs too
// large for LDS, global scratch), split into chunks that fit the workspace,
// and each chunk runs: similarity kernel -> NW kernel (forward, traceback,
// threshold) -> scan -> compaction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/ymine.h"
#include "ym_internal.h"
#include "ym_runtime.h"

using namespace ym;

namespace {
thread_local std::string g_err;
}

namespace ym {

ym_status fail(ym_status code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

ym_status hip_fail(hipError_t e, const char *what) {
  return fail(YM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ------------------------------------------------------------ device buffer
ym_status DevBuf::reserve(size_t bytes, bool exact) {
  if (bytes <= cap) return YM_OK;
  size_t want = exact ? bytes : std::max(bytes, cap * 3 / 2);
  if (ptr) hipFree(ptr);
  ptr = nullptr;
  cap = 0;
  hipError_t e = hipMalloc(&ptr, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    e = hipMalloc(&ptr, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      ptr = nullptr;
      return fail(YM_ENOMEM, "hipMalloc(%zu) failed", bytes);
    }
    want = bytes;
  }
  cap = want;
  return YM_OK;
}

void DevBuf::release() {
  if (ptr) hipFree(ptr);
  ptr = nullptr;
  cap = 0;
}

ym_status HostBuf::reserve(size_t bytes) {
  if (bytes <= cap) return YM_OK;
  if (ptr) hipHostFree(ptr);
  ptr = nullptr;
  cap = 0;
  size_t want = std::max(bytes, size_t(1) << 20);
  hipError_t e = hipHostMalloc(&ptr, want, hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    ptr = nullptr;
    return fail(YM_ENOMEM, "hipHostMalloc(%zu) failed", want);
  }
  cap = want;
  return YM_OK;
}

void HostBuf::release() {
  if (ptr) hipHostFree(ptr);
  ptr = nullptr;
  cap = 0;
}

// ------------------------------------------------------------------ plan
// Per-pair requirement in workspace bytes (score block, scratch, slots).
static inline bool nw_needs_global_dirs(int64_t n, int64_t m) {
  return nw_is_big(n) || n * nw_dir_row_words(m) > kDirLds;
}
// 4-byte words of a pair's direction codes in global scratch: a large pair
// gets 8-byte entries (the persistent-grid sweep tags every word; the
// one-workgroup sweep uses the first half), and every count is even, so every
// pair's words start 8-byte aligned.
static inline int64_t nw_global_dir_words(int64_t n, int64_t m) {
  if (!nw_needs_global_dirs(n, m)) return 0;
  const int64_t w = n * nw_dir_row_words(m);
  return nw_is_big(n) ? 2 * w : (w + 1) & ~int64_t(1);
}
// boundary-row floats in global scratch: one row per strip boundary for the
// pipelined sweep of a large pair (8-byte {H, tag} entries, which the
// persistent-grid sweep needs; the one-workgroup sweep uses the first half),
// one reused row for a one-wave sweep whose row does not fit LDS.  Always
// even, so every pair's rows start 8-byte aligned.
static inline int64_t nw_global_row_floats(int64_t n, int64_t m) {
  if (nw_is_big(n)) return 2 * ((n + 63) / 64 - 1) * (m + 1);
  return (n > 64 && m + 1 > kRowLds) ? ((m + 2) & ~int64_t(1)) : 0;
}
// tickets of a large pair in the persistent-grid sweep (one per strip)
static inline int64_t nw_tickets(int64_t n) { return nw_is_big(n) ? (n + 63) / 64 : 0; }
static inline bool nw_needs_global_row(int64_t n, int64_t m) { return nw_global_row_floats(n, m) > 0; }

// The part of a pair's workspace that the NW kernel writes: its copy is
// needed once per gap penalty swept in one launch.
static size_t pair_nw_bytes(int64_t n, int64_t m) {
  size_t b = 4 /*count*/;
  b += (size_t)nw_global_dir_words(n, m) * 4;
  b += (size_t)nw_global_row_floats(n, m) * 4;
  b += (size_t)std::min(n, m) * 12;
  if (nw_is_big(n)) b += 4 * kNwCtrlPerPair;  // its control words
  return b;
}

size_t pair_bytes(int64_t n, int64_t m, int n_gaps) {
  size_t b = sizeof(PairDesc) + 8 /*moves off*/ + 4 /*NW launch order*/;
  b += (size_t)((n + kMinItemRows - 1) / kMinItemRows) * sizeof(SimItem);  // bound over item sizes
  b += (size_t)score_block(n, m) * 4;
  if (nw_is_big(n)) b += 8 + 4 * nw_tickets(n);  // its entries in the large-pair list, first tickets, ticket map
  b += (size_t)std::max(n_gaps, 1) * pair_nw_bytes(n, m);
  return b;
}


ym_status Chunk::layout(const int64_t *sdo, const int64_t *tdo, int64_t p0_, int64_t p1_, int item_rows_,
                        int n_gaps_) {
  item_rows = item_rows_;
  n_gaps = std::max(n_gaps_, 1);
  p0 = p0_;
  p1 = p1_;
  np = p1 - p0;
  n_items = 0;
  cells = 0;
  s_slots = 0;
  dir_words = 0;
  row_floats = 0;
  slots = 0;
  n_big = 0;
  n_big_strips = 0;
  for (int64_t p = p0; p < p1; p++) {
    const int64_t n = sdo[p + 1] - sdo[p], m = tdo[p + 1] - tdo[p];
    if (n > 0 && m > 0) n_items += (n + item_rows - 1) / item_rows;
    cells += n * m;
    s_slots += score_block(n, m);
    dir_words += nw_global_dir_words(n, m);
    row_floats += nw_global_row_floats(n, m);
    if (nw_is_big(n)) n_big++;
    n_big_strips += nw_tickets(n);
    slots += std::min(n, m);
  }
  // the plan (descriptors, items, move offsets, large-pair list, order) comes
  // first, laid out as in the pinned staging buffer, so one copy uploads it
  size_t o = 0;
  off_descs = o;
  o = align256(o + (size_t)np * sizeof(PairDesc));
  off_items = o;
  o = align256(o + (size_t)std::max<int64_t>(n_items, 1) * sizeof(SimItem));
  off_moves_off = o;
  o = align256(o + (size_t)np * 8);
  off_big = o;
  o = align256(o + (size_t)std::max<int64_t>(n_big, 1) * 4);
  off_order = o;
  o = align256(o + (size_t)std::max<int64_t>(np, 1) * 4);
  off_strip0 = o;
  o = align256(o + (size_t)(n_big + 1) * 4);
  off_tickets = o;
  o = align256(o + (size_t)std::max<int64_t>(n_big_strips, 1) * 4);
  host_bytes = o;
  off_S = o;
  o = align256(o + (size_t)s_slots * 4);
  // the regions the NW kernel writes, one copy per gap penalty of the launch
  // (copy g starts g * its single size further on)
  const size_t G = (size_t)n_gaps;
  off_dirs = o;
  o = align256(o + G * (size_t)dir_words * 4);
  off_rows = o;
  o = align256(o + G * (size_t)row_floats * 4);
  off_ssrc = o;
  o = align256(o + G * (size_t)slots * 4);
  off_stgt = o;
  o = align256(o + G * (size_t)slots * 4);
  off_sscore = o;
  o = align256(o + G * (size_t)slots * 4);
  off_counts = o;
  o = align256(o + G * (size_t)np * 4);
  off_ctrl = o;
  o = align256(o + G * (size_t)(kNwCtrlHead + kNwCtrlPerPair * n_big) * 4);
  bytes = o;
  return YM_OK;
}

// Indices 0..n-1 ordered by key, largest first, equal keys in index order: a
// stable least-significant-digit radix sort (8-bit digits, a pass skipped when
// every key has the same digit).  Launch order only; results never depend on it.
static void order_desc(const uint32_t *key, int64_t n, int32_t *out) {
  std::vector<int32_t> tmp((size_t)n);
  std::vector<uint32_t> k0((size_t)n), k1((size_t)n);
  for (int64_t q = 0; q < n; q++) {
    out[q] = (int32_t)q;
    k0[q] = ~key[q];  // ascending on the complement = descending on the key
  }
  int32_t *a = out, *b = tmp.data();
  uint32_t *ka = k0.data(), *kb = k1.data();
  for (int shift = 0; shift < 32; shift += 8) {
    int64_t cnt[256] = {0};
    for (int64_t q = 0; q < n; q++) cnt[(ka[q] >> shift) & 255]++;
    bool one = false;
    for (int d = 0; d < 256; d++) one |= cnt[d] == n;
    if (one) continue;
    int64_t pos[256], acc = 0;
    for (int d = 0; d < 256; d++) {
      pos[d] = acc;
      acc += cnt[d];
    }
    for (int64_t q = 0; q < n; q++) {
      const int64_t at = pos[(ka[q] >> shift) & 255]++;
      b[at] = a[q];
      kb[at] = ka[q];
    }
    std::swap(a, b);
    std::swap(ka, kb);
  }
  if (a != out) std::memcpy(out, a, (size_t)n * sizeof(int32_t));
}

static inline uint32_t clamp_key(int64_t v) { return v > (int64_t)0xffffffffLL ? 0xffffffffu : (uint32_t)v; }

// Fill descriptors / items / move offsets into pinned host memory.
void Chunk::fill_host(const int64_t *sdo, const int64_t *tdo, char *host) const {
  PairDesc *descs = (PairDesc *)(host + off_descs);
  SimItem *items = (SimItem *)(host + off_items);
  int64_t *moff = (int64_t *)(host + off_moves_off);
  int32_t *big = (int32_t *)(host + off_big);
  int32_t *order = (int32_t *)(host + off_order);
  int64_t s_off = 0, rm_off = 0, out_off = 0, dir_off = 0, row_off = 0, mv = 0, it = 0, nb = 0;
  std::vector<uint32_t> pkey((size_t)np);
  std::vector<int32_t> first_item((size_t)np + 1);
  for (int64_t p = p0; p < p1; p++) {
    const int64_t n = sdo[p + 1] - sdo[p], m = tdo[p + 1] - tdo[p];
    PairDesc &d = descs[p - p0];
    d.src_sent0 = sdo[p];
    d.tgt_sent0 = tdo[p];
    d.s_off = s_off;
    d.rm_off = rm_off;
    d.out_off = out_off;
    d.n = (int32_t)n;
    d.m = (int32_t)m;
    if (nw_needs_global_dirs(n, m)) {
      d.dir_off = dir_off;
      dir_off += nw_global_dir_words(n, m);
    } else {
      d.dir_off = -1;
    }
    if (nw_needs_global_row(n, m)) {
      d.row_off = row_off;
      row_off += nw_global_row_floats(n, m);
    } else {
      d.row_off = -1;
    }
    first_item[p - p0] = (int32_t)it;
    if (n > 0 && m > 0) it += (n + item_rows - 1) / item_rows;
    pkey[p - p0] = clamp_key(n * m);
    moff[p - p0] = mv;
    mv += n + m;
    s_off += score_block(n, m);
    rm_off += n * m;
    out_off += std::min(n, m);
  }
  first_item[np] = (int32_t)it;
  // the largest pairs first in the NW launch, and the largest similarity
  // items (rows x target sentences) first, so each kernel's last workgroups
  // are short ones
  order_desc(pkey.data(), np, order);
  // the large pairs in launch order (largest first); their strips' tickets
  // follow the same order, strip after strip inside a pair
  int32_t *strip0 = (int32_t *)(host + off_strip0);
  int32_t *tickets = (int32_t *)(host + off_tickets);
  int64_t tk = 0;
  for (int64_t q = 0; q < np; q++) {
    const int32_t pq = order[q];
    if (!nw_is_big(descs[pq].n)) continue;
    strip0[nb] = (int32_t)tk;
    for (int64_t k = 0; k < nw_tickets(descs[pq].n); k++) tickets[tk++] = (int32_t)nb;
    big[nb++] = pq;
  }
  strip0[nb] = (int32_t)tk;
  std::vector<uint32_t> ikey((size_t)it);
  std::vector<int32_t> ipair((size_t)it), iorder((size_t)it);
  for (int64_t q = 0; q < np; q++) {
    const int32_t n = descs[q].n, m = descs[q].m;
    for (int32_t k = first_item[q], i0 = 0; k < first_item[q + 1]; k++, i0 += item_rows) {
      ikey[k] = clamp_key((int64_t)(std::min(n, i0 + item_rows) - i0) * m);
      ipair[k] = (int32_t)q;
    }
  }
  order_desc(ikey.data(), it, iorder.data());
  for (int64_t k = 0; k < it; k++) {
    const int32_t src = iorder[k], q = ipair[src];
    const PairDesc &d = descs[q];
    const int32_t i0 = (src - first_item[q]) * item_rows;
    SimItem &x = items[k];
    x.pair = q;
    x.i0 = i0;
    x.i1 = std::min(d.n, i0 + item_rows);
    x.n = d.n;
    x.m = d.m;
    x.pad = 0;
    x.src_sent0 = d.src_sent0;
    x.tgt_sent0 = d.tgt_sent0;
    x.s_off = d.s_off;
    x.rm_off = d.rm_off;
  }
}

}  // namespace ym

// =================================================================== ABI
struct ym_lexicon {
  ym_ctx *ctx = nullptr;  // not dereferenced on free: the context may be gone already
  int device = 0;
  int4 *slots = nullptr;
  int32_t *vals = nullptr;
  uint32_t mask = 0;
  int32_t shift = 0;
  int64_t n_keys = 0, n_pairs = 0;
  int32_t max_fanout = 0;
  int4 *dense = nullptr;  // records of ids 0 .. dense_n - 1 (all keys below kDenseKeys)
  int32_t dense_n = 0;
};

extern "C" {

const char *ym_last_error(void) { return g_err.c_str(); }

const char *ym_version(void) { return "ymine 0.1 (gfx950)"; }

ym_status ym_create(int device, size_t hbm_budget_bytes, ym_ctx **out) {
  if (!out) return fail(YM_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) return fail(YM_EDEVICE, "no HIP device available");
  if (device < 0 || device >= ndev) return fail(YM_EINVAL, "device %d out of range (%d devices)", device, ndev);
  if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  ym_ctx *c = new (std::nothrow) ym_ctx();
  if (!c) return fail(YM_ENOMEM, "context allocation");
  c->device = device;
  {
    const char *v = getenv("YM_SIM_KERNEL");
    c->sim_variant = !v                              ? 1
                     : std::strcmp(v, "tile") == 0   ? 0
                     : std::strcmp(v, "split") == 0  ? 2
                     : std::strcmp(v, "bits") == 0   ? 3
                     : std::strcmp(v, "bits2k") == 0 ? 4
                                                     : 1;
  }
  if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess) {
    delete c;
    return hip_fail(e, "hipStreamCreate");
  }
  if ((e = hipEventCreateWithFlags(&c->stage.done, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&c->ev_ws_free, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&c->ev_up, hipEventDisableTiming)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&c->up_stream, hipStreamNonBlocking)) != hipSuccess) {
    if (c->stage.done) hipEventDestroy(c->stage.done);
    if (c->ev_ws_free) hipEventDestroy(c->ev_ws_free);
    if (c->ev_up) hipEventDestroy(c->ev_up);
    hipStreamDestroy(c->stream);
    delete c;
    return hip_fail(e, "hipEventCreate / hipStreamCreate");
  }
  // the score table, the plan staging buffer and this device's static scratch
  // are set up here, so the allocation-free entry point finds them in place
  ym_status s0 = c->table.reserve((size_t)kTabLen * kTabLen * kTabLen * kTabLen * 4, true);
  if (!s0) s0 = c->stage.buf.reserve(kStagingBytes);
  if (!s0) s0 = static_scratch_init(device);
  if (s0) {
    const std::string msg = ym_last_error();
    ym_destroy(c);
    return fail(s0, "%s", msg.c_str());
  }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = total_b = 0;
  c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.8 * (double)free_b);
  c->arena_limit = std::max<size_t>((size_t)1 << 30, std::min<size_t>((size_t)(0.25 * (double)free_b), (size_t)16 << 30));
  *out = c;
  return YM_OK;
}

void ym_destroy(ym_ctx *c) {
  if (!c) return;
  hipSetDevice(c->device);
  hipStreamSynchronize(c->stream);
  hipStreamSynchronize(c->up_stream);
  for (auto &t : c->ev_pending) {
    hipEventDestroy(t.a);
    hipEventDestroy(t.b);
  }
  for (auto e : c->ev_free) hipEventDestroy(e);
  c->table.release();
  c->in.release();
  c->ws.release();
  c->outb.release();
  c->stage.buf.release();
  c->host_out.release();
  hipEventDestroy(c->stage.done);
  hipEventDestroy(c->ev_ws_free);
  hipEventDestroy(c->ev_up);
  hipStreamDestroy(c->up_stream);
  hipStreamDestroy(c->stream);
  delete c;
}

ym_status ym_lexicon_load(ym_ctx *c, const int32_t *src_ids, const int64_t *off, const int32_t *tgt_ids, int64_t n_src,
                          ym_lexicon **out) {
  if (!c || !out) return fail(YM_EINVAL, "NULL context or out");
  *out = nullptr;
  if (n_src < 0) return fail(YM_EINVAL, "n_src < 0");
  if (n_src > 0 && (!src_ids || !off)) return fail(YM_EINVAL, "NULL lexicon arrays");
  if (n_src > 0 && off[0] != 0) return fail(YM_EINVAL, "off[0] must be 0");
  for (int64_t e = 0; e < n_src; e++) {
    if (off[e + 1] < off[e]) return fail(YM_EINVAL, "lexicon offsets decrease at entry %lld", (long long)e);
    if (src_ids[e] < 0) return fail(YM_EINVAL, "negative source id at entry %lld", (long long)e);
  }
  const int64_t total = n_src > 0 ? off[n_src] : 0;
  if (total > 0 && !tgt_ids) return fail(YM_EINVAL, "NULL tgt_ids");
  if (total >= ((int64_t)1 << 31)) return fail(YM_EINVAL, "lexicon holds 2^31 or more translation pairs");
  for (int64_t v = 0; v < total; v++)
    if (tgt_ids[v] < 0) return fail(YM_EINVAL, "negative target id at value %lld", (long long)v);

  // normalise: sort (key, target), drop duplicates
  std::vector<uint64_t> pr;
  try {
    pr.resize((size_t)total);
  } catch (...) {
    return fail(YM_ENOMEM, "host memory for lexicon");
  }
  int64_t k = 0;
  for (int64_t e = 0; e < n_src; e++)
    for (int64_t v = off[e]; v < off[e + 1]; v++) pr[k++] = ((uint64_t)(uint32_t)src_ids[e] << 32) | (uint32_t)tgt_ids[v];
  std::sort(pr.begin(), pr.end());
  pr.erase(std::unique(pr.begin(), pr.end()), pr.end());
  std::vector<int32_t> keys, cnts, vals(pr.size());
  std::vector<int64_t> offs;
  int32_t maxf = 0;
  for (size_t e = 0; e < pr.size(); e++) {
    const int32_t key = (int32_t)(pr[e] >> 32);
    vals[e] = (int32_t)(uint32_t)pr[e];
    if (keys.empty() || keys.back() != key) {
      keys.push_back(key);
      cnts.push_back(0);
      offs.push_back((int64_t)e);
    }
    cnts.back()++;
    maxf = std::max(maxf, cnts.back());
  }
  if (maxf > YM_MAX_FANOUT) return fail(YM_EINVAL, "a key has %d targets (max %d)", maxf, YM_MAX_FANOUT);

  ym_lexicon *L = new (std::nothrow) ym_lexicon();
  if (!L) return fail(YM_ENOMEM, "lexicon allocation");
  L->ctx = c;
  L->device = c->device;
  L->n_keys = (int64_t)keys.size();
  L->n_pairs = (int64_t)vals.size();
  L->max_fanout = maxf;
  int lg = 10;
  while (((int64_t)1 << lg) < 2 * std::max<int64_t>(L->n_keys, 1)) lg++;
  const int64_t cap = (int64_t)1 << lg;
  L->mask = (uint32_t)(cap - 1);
  L->shift = 32 - lg;

  hipSetDevice(c->device);
  std::lock_guard<std::mutex> lk(c->mu);
  hipError_t e;
  void *dkeys = nullptr, *dcnts = nullptr, *doffs = nullptr;
  auto cleanup = [&]() {
    if (dkeys) hipFree(dkeys);
    if (dcnts) hipFree(dcnts);
    if (doffs) hipFree(doffs);
  };
  if ((e = hipMalloc(&L->slots, (size_t)cap * 2 * sizeof(int4))) != hipSuccess ||
      (e = hipMalloc(&L->vals, std::max<size_t>(vals.size(), 1) * 4)) != hipSuccess ||
      (e = hipMalloc(&dkeys, std::max<size_t>(keys.size(), 1) * 4)) != hipSuccess ||
      (e = hipMalloc(&dcnts, std::max<size_t>(keys.size(), 1) * 4)) != hipSuccess ||
      (e = hipMalloc(&doffs, std::max<size_t>(keys.size(), 1) * 8)) != hipSuccess) {
    (void)hipGetLastError();
    cleanup();
    if (L->slots) hipFree(L->slots);
    if (L->vals) hipFree(L->vals);
    delete L;
    return fail(YM_ENOMEM, "device memory for lexicon");
  }
  e = hipMemsetAsync(L->slots, 0xFF, (size_t)cap * 2 * sizeof(int4), c->stream);  // keys = -1 (empty)
  if (e == hipSuccess && !vals.empty())
    e = hipMemcpyAsync(L->vals, vals.data(), vals.size() * 4, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && !keys.empty()) e = hipMemcpyAsync(dkeys, keys.data(), keys.size() * 4, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && !keys.empty()) e = hipMemcpyAsync(dcnts, cnts.data(), keys.size() * 4, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && !keys.empty()) e = hipMemcpyAsync(doffs, offs.data(), keys.size() * 8, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = launch_lex_insert((const int32_t *)dkeys, (const int32_t *)dcnts, (const int64_t *)doffs, L->vals,
                          (int64_t)keys.size(), L->slots, L->mask, L->shift, c->stream);
  // the dense table, when every key is small (else the batches get a translation pass)
  if (e == hipSuccess && !keys.empty() && keys.back() < kDenseKeys &&
      hipMalloc(&L->dense, (size_t)(keys.back() + 1) * sizeof(int4)) == hipSuccess) {
    L->dense_n = keys.back() + 1;
    e = hipMemsetAsync(L->dense, 0xFF, (size_t)L->dense_n * sizeof(int4), c->stream);  // -1 x 4: no translation
    if (e == hipSuccess)
      e = launch_lex_dense((const int32_t *)dkeys, (const int32_t *)dcnts, (const int64_t *)doffs, L->vals,
                           (int64_t)keys.size(), L->dense, c->stream);
  }
  (void)hipGetLastError();  // a failed dense allocation only means no dense table
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  cleanup();
  if (e != hipSuccess) {
    hipFree(L->slots);
    hipFree(L->vals);
    if (L->dense) hipFree(L->dense);
    delete L;
    return hip_fail(e, "lexicon upload");
  }
  *out = L;
  return YM_OK;
}

void ym_lexicon_free(ym_lexicon *L) {
  if (!L) return;
  hipSetDevice(L->device);
  hipDeviceSynchronize();  // no kernel may still read the table
  hipFree(L->slots);
  hipFree(L->vals);
  if (L->dense) hipFree(L->dense);
  delete L;
}

ym_status ym_profile_enable(ym_ctx *c, int enable) {
  if (!c) return fail(YM_EINVAL, "NULL context");
  std::lock_guard<std::mutex> lk(c->prof_mu);
  c->prof = enable != 0;
  return YM_OK;
}

ym_status ym_profile_read(ym_ctx *c, double ms[4], int64_t launches[4]) {
  if (!c || !ms || !launches) return fail(YM_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(c->prof_mu);
  for (int k = 0; k < 4; k++) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  hipSetDevice(c->device);
  for (auto &t : c->ev_pending) {
    float x = 0.0f;
    hipError_t e = hipEventSynchronize(t.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&x, t.a, t.b);
    if (e != hipSuccess) return hip_fail(e, "profile read");
    if (t.kind >= 0 && t.kind < 4) {
      ms[t.kind] += x;
      launches[t.kind]++;
    }
    c->ev_free.push_back(t.a);
    c->ev_free.push_back(t.b);
  }
  c->ev_pending.clear();
  return YM_OK;
}

ym_status ym_check_pair(int64_t n, int64_t m) { return check_pair_shape(n, m, 0); }

ym_status ym_set_wait_limit(ym_ctx *c, int64_t ticks) {
  if (!c) return fail(YM_EINVAL, "NULL context");
  std::lock_guard<std::mutex> lk(c->mu);
  c->nw_wait_ticks = ticks < 0 ? kNwWaitTicks : (uint64_t)ticks;
  return YM_OK;
}

ym_status ym_lexicon_stats(const ym_lexicon *L, int64_t *n_keys, int64_t *n_pairs, int32_t *max_fanout) {
  if (!L) return fail(YM_EINVAL, "NULL lexicon");
  if (n_keys) *n_keys = L->n_keys;
  if (n_pairs) *n_pairs = L->n_pairs;
  if (max_fanout) *max_fanout = L->max_fanout;
  return YM_OK;
}

}  // extern "C"

// ------------------------------------------------------- shared internals
namespace ym {

LexDev lex_dev(const ym_lexicon *L) {
  LexDev d;
  d.slots = L->slots;
  d.vals = L->vals;
  d.mask = L->mask;
  d.shift = L->shift;
  d.dense = L->dense;
  d.dense_n = L->dense_n;
  return d;
}

ym_status check_params(const ym_params *p) {
  if (!p) return fail(YM_EINVAL, "NULL params");
  for (int k = 0; k < 4; k++)
    if (!std::isfinite(p->w[k])) return fail(YM_EINVAL, "weight %d is not finite", k);
  if (!std::isfinite(p->gap)) return fail(YM_EINVAL, "gap is not finite");
  if (!std::isfinite(p->threshold)) return fail(YM_EINVAL, "threshold is not finite");
  return YM_OK;
}

// Make sure the score table matches the weights (rebuilt on change).
ym_status ensure_table(ym_ctx *c, const ym_params *p, hipStream_t st) {
  if (c->table_valid && std::memcmp(c->table_w, p->w, sizeof c->table_w) == 0) return YM_OK;
  ym_status s = c->table.reserve((size_t)kTabLen * kTabLen * kTabLen * kTabLen * 4);
  if (s) return s;
  hipError_t e = launch_score_table(p->w[0], p->w[1], p->w[2], p->w[3], (float *)c->table.ptr, st);
  if (e != hipSuccess) return hip_fail(e, "score table");
  std::memcpy(c->table_w, p->w, sizeof c->table_w);
  c->table_valid = true;
  return YM_OK;
}

ym_status translate_batch(ym_ctx *c, const ym_lexicon *L, DevBatch &b, char *head, hipStream_t st) {
  b.trans = (const int4 *)head;
  hipError_t e;
  {
    KernelTimer kt(c, 3, st);
    e = launch_translate(b.src_tok, b.n_src_tok, lex_dev(L), (int4 *)head, st);
  }
  return e == hipSuccess ? YM_OK : hip_fail(e, "translate kernel");
}

// Validate a host pair table: offsets start at 0 and never decrease.
ym_status check_doc_off(const int64_t *o, int64_t n_pairs, const char *what) {
  if (!o) return fail(YM_EINVAL, "%s is NULL", what);
  if (o[0] != 0) return fail(YM_EINVAL, "%s[0] must be 0", what);
  for (int64_t p = 0; p < n_pairs; p++) {
    if (o[p + 1] < o[p]) return fail(YM_EINVAL, "%s decreases at pair %lld", what, (long long)p);
    if (o[p + 1] - o[p] > 0x7fffffffLL) return fail(YM_EINVAL, "%s: pair %lld has 2^31 sentences or more", what, (long long)p);
  }
  return YM_OK;
}

ym_status check_pair_shape(int64_t n, int64_t m, int64_t pair) {
  if (n < 0 || m < 0) return fail(YM_EINVAL, "pair %lld: negative sentence count", (long long)pair);
  if (n > kMaxDocSents || m > kMaxDocSents)
    return fail(YM_EINVAL, "pair %lld: a document has more than %lld sentences", (long long)pair, (long long)kMaxDocSents);
  if (score_slots(n, m) > kMaxPairSlots)
    return fail(YM_EINVAL, "pair %lld: %lld x %lld sentences need %lld score slots (at most 2^31 - 4)", (long long)pair,
                (long long)n, (long long)m, (long long)score_slots(n, m));
  return YM_OK;
}

// Plan bytes of one pair (the part of pair_bytes that is uploaded from the
// host: descriptor, similarity items, move offset, large-pair entry, NW order).
static size_t pair_plan_bytes(int64_t n, int64_t m) {
  (void)m;
  return sizeof(PairDesc) + (size_t)((n + kMinItemRows - 1) / kMinItemRows) * sizeof(SimItem) + 8 + 4 +
         (nw_is_big(n) ? 8 + 4 * nw_tickets(n) : 0);
}
static const size_t kPlanSlack = 8 * 256;  // alignment padding of the plan's seven regions, and their minimum sizes

// Split pairs [0, n_pairs) into chunks whose workspace fits `ws_bytes` and,
// when `plan_cap` is not 0, whose plan fits `plan_cap` bytes.
ym_status plan_chunks(const int64_t *sdo, const int64_t *tdo, int64_t n_pairs, size_t ws_bytes,
                      std::vector<std::pair<int64_t, int64_t>> &chunks, size_t plan_cap, int n_gaps) {
  chunks.clear();
  int64_t p = 0;
  for (int64_t q = 0; q < n_pairs; q++) {
    const ym_status st = check_pair_shape(sdo[q + 1] - sdo[q], tdo[q + 1] - tdo[q], q);
    if (st) return st;
  }
  while (p < n_pairs) {
    size_t acc = chunk_fixed_bytes(n_gaps), plan = kPlanSlack;
    int64_t q = p;
    while (q < n_pairs) {
      const int64_t n = sdo[q + 1] - sdo[q], m = tdo[q + 1] - tdo[q];
      const size_t b = pair_bytes(n, m, n_gaps), h = plan_cap ? pair_plan_bytes(n, m) : 0;
      if (q > p && (acc + b > ws_bytes || (plan_cap && plan + h > plan_cap))) break;
      acc += b;
      plan += h;
      q++;
    }
    if (acc > ws_bytes) return fail(YM_ENOMEM, "pair %lld needs %zu workspace bytes, %zu given", (long long)p, acc, ws_bytes);
    if (plan_cap && plan > plan_cap)
      return fail(YM_ENOMEM, "pair %lld needs %zu plan bytes, %zu available", (long long)p, plan, plan_cap);
    chunks.push_back({p, q});
    p = q;
  }
  return YM_OK;
}

// Enqueue one chunk: upload its plan, then the four kernels.
ym_status upload_plan(ym_ctx *c, const int64_t *sdo, const int64_t *tdo, const Chunk &ch, char *ws, hipStream_t st,
                      Staging *stg, bool side) {
  // plan -> pinned staging -> workspace (wait for the previous upload to have left the staging buffer)
  if (!stg) stg = &c->stage;
  hipError_t e = stg->caller_syncs ? hipSuccess : hipEventSynchronize(stg->done);
  if (e != hipSuccess) return hip_fail(e, "staging wait");
  ym_status s = stg->buf.reserve(ch.host_bytes);
  if (s) return s;
  ch.fill_host(sdo, tdo, (char *)stg->buf.ptr);
  // the whole plan in one copy (same layout on both sides); on the upload
  // stream once the work already on `st` (which may read the previous plan)
  // is done.  When the work is captured into a graph the caller records
  // stg->done after launching it.
  hipStream_t us = st;
  if (side) {
    if ((e = hipEventRecord(c->ev_ws_free, st)) != hipSuccess || (e = hipStreamWaitEvent(c->up_stream, c->ev_ws_free, 0)))
      return hip_fail(e, "plan upload order");
    us = c->up_stream;
  }
  if ((e = hipMemcpyAsync(ws + ch.off_descs, stg->buf.ptr, ch.host_bytes, hipMemcpyHostToDevice, us)) != hipSuccess ||
      (!stg->caller_syncs && (e = hipEventRecord(stg->done, us)) != hipSuccess) ||
      (side && (e = hipEventRecord(c->ev_up, us)) != hipSuccess))
    return hip_fail(e, "plan upload");
  return YM_OK;
}

ym_status run_chunk(ym_ctx *c, const ym_lexicon *L, const DevBatch &b, const ym_params *prm, const int64_t *sdo,
                    const int64_t *tdo, const Chunk &ch, char *ws, const ym_device_out &out, hipStream_t st,
                    const DebugOut *dbg, Staging *stg, bool plan_ready) {
  hipError_t e;
  ym_status s;
  if (!plan_ready && (s = upload_plan(c, sdo, tdo, ch, ws, st, stg, false))) return s;

  const PairDesc *descs = (const PairDesc *)(ws + ch.off_descs);
  float *S = (float *)(ws + ch.off_S);  // strip-diagonal layout
  if (dbg && dbg->reuse_S) {
    // scores computed by an earlier run of this chunk
  } else if (dbg && dbg->S_rowmajor_in) {
    if ((e = launch_relayout(descs, ch.np, dbg->S_rowmajor_in, S, 1, st)) != hipSuccess) return hip_fail(e, "relayout");
  } else {
    SimArgs a;
    a.items = (const SimItem *)(ws + ch.off_items);
    a.n_items = ch.n_items;
    a.descs = descs;
    a.src_sent_off = b.src_sent_off;
    a.src_tok = b.src_tok;
    a.tgt_sent_off = b.tgt_sent_off;
    a.tgt_tok = b.tgt_tok;
    a.n_src_sent = b.n_src_sent;
    a.n_tgt_sent = b.n_tgt_sent;
    a.n_src_tok = b.n_src_tok;
    a.n_tgt_tok = b.n_tgt_tok;
    a.lex = lex_dev(L);
    a.trans = b.trans;
    a.w0 = prm->w[0];
    a.w1 = prm->w[1];
    a.w2 = prm->w[2];
    a.w3 = prm->w[3];
    a.table = (const float *)c->table.ptr;
    a.S = S;
    a.ms_out = dbg ? dbg->ms : nullptr;
    a.mt_out = dbg ? dbg->mt : nullptr;
    const int grid = (int)std::min<int64_t>(ch.n_items, (int64_t)1 << 30);
    {
      KernelTimer kt(c, 0, st);
      e = launch_similarity(a, grid, c->sim_variant, st);
    }
    if (e != hipSuccess) return hip_fail(e, "similarity kernel");
    if (dbg && dbg->S_rowmajor_out &&
        (e = launch_relayout(descs, ch.np, S, dbg->S_rowmajor_out, 0, st)) != hipSuccess)
      return hip_fail(e, "relayout");
    if (dbg && dbg->sim_only) return YM_OK;
  }
  NwArgs n;
  n.descs = descs;
  n.n_pairs = ch.np;
  n.S = S;
  n.gap = prm->gap;
  n.tau = prm->threshold;
  n.dir_scratch = (uint32_t *)(ws + ch.off_dirs);
  n.row_scratch = (float *)(ws + ch.off_rows);
  n.slot_src = (int32_t *)(ws + ch.off_ssrc);
  n.slot_tgt = (int32_t *)(ws + ch.off_stgt);
  n.slot_score = (float *)(ws + ch.off_sscore);
  n.counts = (int32_t *)(ws + ch.off_counts);
  n.align = out.align_score;
  n.pair_base = ch.p0;
  n.moves = dbg ? dbg->moves_dev : nullptr;
  n.moves_off = (const int64_t *)(ws + ch.off_moves_off);
  n.big = (const int32_t *)(ws + ch.off_big);
  n.order = (const int32_t *)(ws + ch.off_order);
  n.n_big = ch.n_big;
  n.n_moves = dbg ? dbg->n_moves_dev : nullptr;
  n.wait_ticks = c->nw_wait_ticks;
  n.status = out.status;
  n.split = c->nw_large;
  n.big_strip0 = (const int32_t *)(ws + ch.off_strip0);
  n.ticket_big = (const int32_t *)(ws + ch.off_tickets);
  n.n_big_strips = ch.n_big_strips;
  n.ctrl = (int32_t *)(ws + ch.off_ctrl);
  if (dbg && dbg->gaps) {  // every gap of a sweep in this one launch, outputs per gap
    n.gaps = dbg->gaps;
    n.n_gaps = ch.n_gaps;
    n.g_dirs = ch.dir_words;
    n.g_rows = ch.row_floats;
    n.g_slots = ch.slots;
    n.g_counts = ch.np;
    n.g_align = dbg->align_stride;
    n.g_ctrl = kNwCtrlHead + (int64_t)kNwCtrlPerPair * ch.n_big;
  }
  if (n.moves) n.moves += dbg->moves_base;
  {
    KernelTimer kt(c, 1, st);
    e = launch_nw(n, c->nw_pairs_per_group, st);
  }
  if (e != hipSuccess) return hip_fail(e, "nw kernel");
  if (dbg && dbg->gaps) return YM_OK;  // a gap sweep counts from the per-pair slots itself
  {
    KernelTimer kt(c, 2, st);
    e = launch_scan(n.counts, ch.np, out.pair_off + ch.p0, ch.p0 == 0, st);
    if (e == hipSuccess)
      e = launch_compact(descs, ch.np, n.counts, out.pair_off + ch.p0, n.slot_src, n.slot_tgt, n.slot_score, out.src_idx,
                         out.tgt_idx, out.score, st);
  }
  if (e != hipSuccess) return hip_fail(e, "scan / compact");
  return YM_OK;
}

}  // namespace ym
