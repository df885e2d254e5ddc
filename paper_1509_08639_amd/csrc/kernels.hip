// Device kernels of libymine for gfx950 (CDNA4, wave64).
//
//   lex_insert_kernel,
//   lex_dense_kernel     build the HBM-resident lexicon hash and, for small
//                        key ranges, the dense record table (session setup)
//   score_table_kernel   sentence-pair score for every (a, b, m_s, m_t) with
//                        a, b < 64, from the current classifier weights
//   translate_kernel     translation record of every source token of a batch
//   sim_kernel,
//   sim_tile_kernel,
//   sim_bits_kernel      (a) sentence-pair score matrix of each document pair
//   nw_kernel,
//   nw_big_kernel        (b) Needleman-Wunsch forward pass, traceback and
//                        threshold filter of each document pair
//   scan_kernel,
//   compact_kernel       per-pair counts -> CSR offsets, slot -> CSR copy
//   tune_count_kernel,
//   merge_bi_kernel      parameter sweep counts; bidirectional union
//   relayout_kernel      row-major <-> strip-diagonal scores (parity entries)
//
// Floating point: the score is built from correctly rounded float divides,
// products and sums in a fixed order (no contraction; built with
// -ffp-contract=off and explicit __f*_rn), and the logistic is evaluated in
// double and rounded once.  The DP uses only float additions and strict
// comparisons.  Denormals are preserved.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "ym_internal.h"

namespace ym {

__device__ __forceinline__ uint32_t hash32(int32_t x) { return (uint32_t)x * 0x9E3779B1u; }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Make one wave's global and LDS writes visible to its own later reads (a
// one-wave workgroup: workgroup scope, no device-wide cache write-back).
__device__ __forceinline__ void wave_sync_mem() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// ------------------------------------------------------------------ score
// Section 4: the classifier's confidence is a probability.  Features are the
// lexicon-overlap fractions f1 = m_s/a, f2 = m_t/b and the length ratio
// f3 = min/max; z = ((w0 + w1 f1) + w2 f2) + w3 f3; S = 1 / (1 + e^-z).
__device__ __forceinline__ float ratio_rn(int num, int den) {
  return den == 0 ? 0.0f : __fdiv_rn((float)num, (float)den);
}

__device__ __noinline__ float score_direct(float w0, float w1, float w2, float w3, int ms, int a, int mt, int b) {
  const float f1 = ratio_rn(ms, a);
  const float f2 = ratio_rn(mt, b);
  const float f3 = ratio_rn(a < b ? a : b, a < b ? b : a);
  float z = __fadd_rn(w0, __fmul_rn(w1, f1));
  z = __fadd_rn(z, __fmul_rn(w2, f2));
  z = __fadd_rn(z, __fmul_rn(w3, f3));
  const double e = exp(-(double)z);
  return (float)(1.0 / (1.0 + e));
}

// Index of the score of (ms, a, mt, b) in the score table:
// ((ms * L + mt) * L + a) * L + b with L = kTabLen.  The overlap counts are the
// outer indices, so the cells of the common small counts (most sentence pairs
// share a few words at most) read a few 16 KB planes that stay in L2.
__device__ __forceinline__ int tab_index(int a, int b, int ms, int mt) {
  return (((ms << kLogTabLen) | mt) << (2 * kLogTabLen)) | (a << kLogTabLen) | b;
}

__global__ __launch_bounds__(256) void score_table_kernel(float w0, float w1, float w2, float w3, float *table) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  constexpr int M = kTabLen - 1, B = kLogTabLen;
  const int b = idx & M, a = (idx >> B) & M, mt = (idx >> (2 * B)) & M, ms = (idx >> (3 * B)) & M;
  table[idx] = (ms <= a && mt <= b) ? score_direct(w0, w1, w2, w3, ms, a, mt, b) : 0.0f;
}

// ---------------------------------------------------------------- lexicon
// Lexicon slot h is two int4: {key, count, offset, -1} and the key's
// translation record: up to four target ids inline (-1 padded), or
// {-2, offset, count, 0} for a key with more than four (read from the value
// array when used).
// A key's translation record: its targets inline (-1 padded) when it has at
// most four, else {-2, offset, count, 0} into the value array.
__device__ __forceinline__ int4 lex_record(int c, int32_t o, const int32_t *vals) {
  int4 r = make_int4(-1, -1, -1, -1);
  if (c > 4) {
    r = make_int4(-2, o, c, 0);
  } else {
    if (c > 0) r.x = vals[o];
    if (c > 1) r.y = vals[o + 1];
    if (c > 2) r.z = vals[o + 2];
    if (c > 3) r.w = vals[o + 3];
  }
  return r;
}

// The dense table: record of key k at index k (other ids keep -1 x 4).
__global__ __launch_bounds__(256) void lex_dense_kernel(const int32_t *keys, const int32_t *cnts, const int64_t *offs,
                                                        const int32_t *vals, int64_t n, int4 *dense) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < n) dense[keys[k]] = lex_record(cnts[k], (int32_t)offs[k], vals);
}

__global__ __launch_bounds__(256) void lex_insert_kernel(const int32_t *keys, const int32_t *cnts,
                                                         const int64_t *offs, const int32_t *vals, int64_t n,
                                                         int4 *slots, uint32_t mask, int shift) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  const int32_t key = keys[k];
  uint32_t h = hash32(key) >> shift;
  for (;;) {  // load factor <= 1/2 and distinct keys: an empty slot is always reached
    const int prev = atomicCAS(&slots[2 * h].x, kEmpty, key);
    if (prev == kEmpty) {
      const int c = cnts[k];
      const int32_t o = (int32_t)offs[k];
      slots[2 * h].y = c;
      slots[2 * h].z = o;
      slots[2 * h + 1] = lex_record(c, o, vals);
      return;
    }
    h = (h + 1) & mask;
  }
}

// Translations of every source token of a batch, resolved once per call
// (the key's record; -1 x 4 for ids that are not keys): one read of the
// lexicon's dense table when it has one, else a hash lookup.  Each thread
// takes four tokens 256 apart, so four independent reads or probe chains are
// in flight.
constexpr int kTransPerThread = 4;
__global__ __launch_bounds__(256) void translate_kernel(const int32_t *tok, int64_t n, LexDev L, int4 *out) {
  const int64_t base = (int64_t)blockIdx.x * (256 * kTransPerThread) + threadIdx.x;
  if (L.dense) {
    int32_t y[kTransPerThread];
#pragma unroll
    for (int u = 0; u < kTransPerThread; u++) {
      const int64_t k = base + 256 * u;
      y[u] = k < n ? tok[k] : -1;
    }
    int4 r[kTransPerThread];
#pragma unroll
    for (int u = 0; u < kTransPerThread; u++)
      r[u] = (y[u] >= 0 && y[u] < L.dense_n) ? L.dense[y[u]] : make_int4(-1, -1, -1, -1);
#pragma unroll
    for (int u = 0; u < kTransPerThread; u++) {
      const int64_t k = base + 256 * u;
      if (k < n) out[k] = r[u];
    }
    return;
  }
  int32_t x[kTransPerThread];
  uint32_t h[kTransPerThread];
  int4 s[kTransPerThread], t[kTransPerThread];
  bool more[kTransPerThread];
#pragma unroll
  for (int u = 0; u < kTransPerThread; u++) {
    const int64_t k = base + 256 * u;
    x[u] = k < n ? tok[k] : -1;
  }
#pragma unroll
  for (int u = 0; u < kTransPerThread; u++) {
    h[u] = hash32(x[u]) >> L.shift;
    if (x[u] >= 0) {
      s[u] = L.slots[2 * h[u]];
      t[u] = L.slots[2 * h[u] + 1];
    } else {
      s[u] = make_int4(kEmpty, 0, 0, 0);
      t[u] = make_int4(-1, -1, -1, -1);
    }
  }
#pragma unroll
  for (int u = 0; u < kTransPerThread; u++) {
    more[u] = x[u] >= 0 && s[u].x != x[u] && s[u].x != kEmpty;
    while (more[u]) {  // collision: next slot
      h[u] = (h[u] + 1) & L.mask;
      s[u] = L.slots[2 * h[u]];
      t[u] = L.slots[2 * h[u] + 1];
      more[u] = s[u].x != x[u] && s[u].x != kEmpty;
    }
  }
#pragma unroll
  for (int u = 0; u < kTransPerThread; u++) {
    const int64_t k = base + 256 * u;
    if (k < n) out[k] = (x[u] >= 0 && s[u].x == x[u]) ? t[u] : make_int4(-1, -1, -1, -1);
  }
}

// ---------------------------------------------------------- LDS id table
__device__ __forceinline__ int u_insert(int32_t *ukey, int32_t x) {
  uint32_t h = hash32(x) >> (32 - kLogUcap);
  for (;;) {  // at most kTcap distinct keys in kUcap slots
    const int prev = atomicCAS(&ukey[h], kEmpty, x);
    if (prev == kEmpty || prev == x) return (int)h;
    h = (h + 1) & (kUcap - 1);
  }
}

__device__ __forceinline__ int u_find(const int32_t *ukey, int32_t x) {
  if (x < 0) return -1;
  uint32_t h = hash32(x) >> (32 - kLogUcap);
  for (;;) {
    const int k = ukey[h];
    if (k == x) return (int)h;
    if (k == kEmpty) return -1;
    h = (h + 1) & (kUcap - 1);
  }
}

// OR `bits` into the word of every translation of one source token that is an
// id of the staged chunk.
__device__ __forceinline__ void scatter_token(const int4 t4, uint32_t bits, const int32_t *ukey,
                                              const uint16_t *ulid, uint32_t *Mw, const int32_t *vals) {
  if (t4.x == -2) {
    for (int e = 0; e < t4.z; e++) {
      const int s = u_find(ukey, vals[t4.y + e]);
      if (s >= 0) atomicOr(&Mw[ulid[s]], bits);
    }
  } else {
    const int s0 = u_find(ukey, t4.x), s1 = u_find(ukey, t4.y), s2 = u_find(ukey, t4.z), s3 = u_find(ukey, t4.w);
    if (s0 >= 0) atomicOr(&Mw[ulid[s0]], bits);
    if (s1 >= 0) atomicOr(&Mw[ulid[s1]], bits);
    if (s2 >= 0) atomicOr(&Mw[ulid[s2]], bits);
    if (s3 >= 0) atomicOr(&Mw[ulid[s3]], bits);
  }
}

// Exclusive prefix sum over the 256 threads of a block.
__device__ __forceinline__ int block_excl_sum256(int v, int *sh, int *total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wv] = x;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kSimWaves; w++) {
    const int s = sh[w];
    base += (w < wv) ? s : 0;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

__device__ __forceinline__ int64_t clamp64(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ float shift_up_one_lane(float v) {
  // wave_shr:1 -- lane l receives lane l-1's value (lane 0 keeps its own)
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x138, 0xF, 0xF, false));
}


// End of the target chunk starting at sentence j0, by the first wave: the
// largest j1 <= j0 + 64 whose sentences [j0, j1) hold at most kTcap tokens
// (at least one sentence).  Lane L tests j1 = j0 + 1 + L, all in one round of
// loads; the chunk ends before the first candidate that does not fit.  With
// `ends`, lane L also keeps the end of the chunk's sentence L relative to the
// chunk's first token (clamped to [0, 2^30]).
__device__ __forceinline__ void chunk_end(const int64_t *toffs, int j0, int m, int64_t n_tok, int *out, int *ends) {
  const int lane = threadIdx.x & 63;
  const int64_t base = clamp64(toffs[j0], 0, n_tok);
  const int jj = j0 + 1 + lane;
  const bool ok = jj <= min(m, j0 + kJcap);
  const int64_t e = ok ? clamp64(toffs[jj], 0, n_tok) - base : 0;
  const uint64_t bal = __ballot(ok && e <= kTcap);
  const int lead = ~bal == 0 ? 64 : __builtin_ctzll(~bal);  // candidates that fit, from the first on
  if (lane == 0) *out = j0 + max(1, lead);
  if (ends) ends[lane] = (int)clamp64(e, 0, 1 << 30);
}

// ------------------------------------------------------ (a) similarity
// One work item = (pair, source sentences [i0, i1)).  Target sentences are
// taken in chunks of at most 64 sentences and kTcap tokens.  Each chunk's
// distinct target ids get dense local ids through an LDS hash, and the
// chunk's tokens are restaged in LDS as local ids (each sentence padded to a
// multiple of 4 with id 0).  Lane jj of every wave owns target sentence jj of
// the chunk and keeps the LDS addresses of its first 32 ids in registers for
// the whole chunk.  A wave then takes one source sentence i at a time: it
// marks, in an LDS word per local id, which source positions q translate to
// that id (bit q) and whether the id is in X_i (top bit, word 0 stays 0), and
// every lane walks its sentence's words:
//   m_t = number of tokens whose word has the top bit,
//   m_s = popcount of the OR of the words' position bits.
// Two source sentences of at most 31 tokens share a step (one 32-bit word
// each in an 8-byte entry); a longer one takes a step of its own with the
// entry as one 64-bit word (63 positions per pass; further passes for longer
// sentences carry position bits only).
constexpr int kRegTok = 32;  // target ids per lane held as register addresses

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// DPP lane moves: quad_perm [1,0,3,2] (0xB1), [2,3,0,1] (0x4E), mirror
// inside 8 lanes (0x141), mirror inside 16 lanes (0x140)
template <int kCtrl>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, kCtrl, 0xF, 0xF, false);
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// 8-byte LDS read at a 32-bit LDS byte address (the addresses held in
// registers already include the array's base, so no add per read)
typedef __attribute__((address_space(3))) const unsigned long long lds_cu64;
__device__ __forceinline__ uint2 lds_u2_at(uint32_t addr) {
  const unsigned long long v = *(lds_cu64 *)(uintptr_t)addr;
  return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
}

// LDS hash entry of the lanes kernel: key and its dense local id side by
// side, so a lookup is one 8-byte read.  Insert target id x (>= 0): its
// slot, and whether x was new to the table.
__device__ __forceinline__ int u2_insert_fresh(int2 *ent, int32_t x, bool &fresh) {
  uint32_t h = hash32(x) >> (32 - kLogUcap);
  for (;;) {  // at most kTcap distinct keys in kUcap slots
    const int prev = atomicCAS(&ent[h].x, kEmpty, x);
    if (prev == kEmpty || prev == x) {
      fresh = prev == kEmpty;
      return (int)h;
    }
    h = (h + 1) & (kUcap - 1);
  }
}

// local id of target id x in the chunk, 0 if x is not one of its ids
__device__ __forceinline__ int u2_lid(const int2 *ent, int32_t x) {
  if (x < 0) return 0;
  uint32_t h = hash32(x) >> (32 - kLogUcap);
  int2 e = ent[h];
  while (e.x != x && e.x != kEmpty) {
    h = (h + 1) & (kUcap - 1);
    e = ent[h];
  }
  return e.x == x ? e.y : 0;
}

// local ids of four keys at once: the four first probes are issued together
__device__ __forceinline__ int4 u2_lid4(const int2 *ent, const int4 x) {
  constexpr uint32_t kMask = kUcap - 1;
  uint32_t h0 = hash32(x.x) >> (32 - kLogUcap), h1 = hash32(x.y) >> (32 - kLogUcap);
  uint32_t h2 = hash32(x.z) >> (32 - kLogUcap), h3 = hash32(x.w) >> (32 - kLogUcap);
  int2 e0 = ent[h0], e1 = ent[h1], e2 = ent[h2], e3 = ent[h3];
  bool p0 = x.x >= 0 && e0.x != x.x && e0.x != kEmpty, p1 = x.y >= 0 && e1.x != x.y && e1.x != kEmpty;
  bool p2 = x.z >= 0 && e2.x != x.z && e2.x != kEmpty, p3 = x.w >= 0 && e3.x != x.w && e3.x != kEmpty;
  while (p0 || p1 || p2 || p3) {
    if (p0) {
      h0 = (h0 + 1) & kMask;
      e0 = ent[h0];
      p0 = e0.x != x.x && e0.x != kEmpty;
    }
    if (p1) {
      h1 = (h1 + 1) & kMask;
      e1 = ent[h1];
      p1 = e1.x != x.y && e1.x != kEmpty;
    }
    if (p2) {
      h2 = (h2 + 1) & kMask;
      e2 = ent[h2];
      p2 = e2.x != x.z && e2.x != kEmpty;
    }
    if (p3) {
      h3 = (h3 + 1) & kMask;
      e3 = ent[h3];
      p3 = e3.x != x.w && e3.x != kEmpty;
    }
  }
  return make_int4(x.x >= 0 && e0.x == x.x ? e0.y : 0, x.y >= 0 && e1.x == x.y ? e1.y : 0,
                   x.z >= 0 && e2.x == x.z ? e2.y : 0, x.w >= 0 && e3.x == x.w ? e3.y : 0);
}

__device__ __forceinline__ int64_t readlane64(int64_t v, int k) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, k);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), k);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

static_assert(kMaxItemRows / kSimWaves <= 64, "one lane per row of a wave");
constexpr int kQuadBits = 15;  // source positions per 16-bit field of a four-row step (bit 15: hit bit)

// kHelp: chunks holding target sentences of more than 32 tokens use the lanes
// they leave over to split the reads (below).  A separate instantiation,
// because the extra code costs registers in the common short-sentence case.
template <bool kHelp>
__global__ __launch_bounds__(kSimThreads, 3) void sim_kernel(SimArgs a) {
  __shared__ int2 uent[kUcap];
  __shared__ __align__(16) uint16_t tdoc[kTdocCap];
  __shared__ uint16_t toff[kJcap];        // start of sentence jj in the padded staging
  __shared__ uint16_t toff_o[kJcap + 1];  // start of sentence jj in the chunk's token range
  __shared__ uint16_t tlen[kJcap];
  __shared__ __align__(16) uint2 Mw2[kSimWaves][kTcap + 4];  // per wave and local id: two mask words
  __shared__ int sh_scan[kSimWaves];
  __shared__ int sh_j1;
  __shared__ int sh_ends[kJcap];  // chunk's sentence ends, relative to its first token
  __shared__ int sh_nlid, sh_npad;  // chunk's distinct ids, padded staging length
  __shared__ uint8_t sh_own[kSimWaves][64];  // helper layout: sentence read by each lane

  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  uint32_t *Mx = reinterpret_cast<uint32_t *>(Mw2[wv]);
  const uint32_t mw_lds = (uint32_t)(uintptr_t)&Mw2[0][0];  // LDS byte address of the masks

  // The mask words start at zero once; every step clears what it set (the
  // one-row path clears all the chunk's entries), so they are zero again at
  // the start of every step and chunk.
  for (int k = tid; k < kSimWaves * (kTcap + 4) / 2; k += kSimThreads)
    reinterpret_cast<uint4 *>(&Mw2[0][0])[k] = make_uint4(0, 0, 0, 0);
  __syncthreads();

  for (int64_t item = blockIdx.x; item < a.n_items; item += gridDim.x) {
    const SimItem it = a.items[item];
    PairDesc d;  // the descriptor fields the item carries
    d.n = it.n, d.m = it.m, d.src_sent0 = it.src_sent0, d.tgt_sent0 = it.tgt_sent0, d.s_off = it.s_off, d.rm_off = it.rm_off;
    const int n = d.n, m = d.m;
    if (m <= 0 || it.i1 <= it.i0) continue;
    const int64_t *toffs = a.tgt_sent_off + d.tgt_sent0;
    const int64_t *soffs = a.src_sent_off + d.src_sent0;
    // This wave's source rows are rows i0 + 2 wv + 8 q and the row after (q =
    // 0, 1, ...; items start on 64-row strips, so the two are adjacent).
    // Kernel 1 takes them in that order, two per step (a longer row alone).
    // Kernel 2 first orders them by length class: rows of at most 15 tokens
    // go four to a step (a 16-bit field each in the 8-byte mask entry: 15
    // position bits and the hit bit), rows of 16-31 tokens two to a step (a
    // 32-bit field each), longer rows one to a step (the whole entry).  Lane k
    // holds wave-row k: its first token, and its length (saturated at 2^24 -
    // 1) | (row - i0) << 24.
    const int nrows = 2 * ((it.i1 - it.i0) / (2 * kSimWaves)) + min(2, max(0, (it.i1 - it.i0) % (2 * kSimWaves) - 2 * wv));
    int64_t rsb = 0;
    int rinf = 0;
    int nQ = 0, nP = nrows, nL = 0;  // wave-rows [0, nQ) four per step, then nP two per step, then nL alone
    {
      const int row = it.i0 + 2 * wv + 2 * kSimWaves * (lane >> 1) + (lane & 1);
      int64_t sb = 0, len = 0;
      if (lane < nrows) {
        sb = clamp64(soffs[row], 0, a.n_src_tok);
        len = clamp64(soffs[row + 1], sb, a.n_src_tok) - sb;
      }
      if constexpr (kHelp) {
        const int inf = (int)min(len, (int64_t)0xFFFFFF) | ((row - it.i0) << 24);
        const int cls = lane >= nrows ? 3 : len <= kQuadBits ? 0 : len <= kPosBits ? 1 : 2;
        const uint64_t mQ = __ballot(cls == 0), mP = __ballot(cls == 1), mL = __ballot(cls == 2);
        nQ = __popcll(mQ), nP = __popcll(mP), nL = __popcll(mL);
        const uint64_t below = (1ull << lane) - 1;
        const int dst = cls == 0 ? __popcll(mQ & below)
                      : cls == 1 ? nQ + __popcll(mP & below)
                      : cls == 2 ? nQ + nP + __popcll(mL & below)
                                 : lane;  // a permutation of the 64 lanes
        const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_permute(dst << 2, (int)(uint32_t)sb);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_permute(dst << 2, (int)(uint32_t)(sb >> 32));
        rsb = (int64_t)(((uint64_t)hi << 32) | lo);
        rinf = __builtin_amdgcn_ds_permute(dst << 2, inf);
      } else {  // kernel 1: lane k holds row k's first token and length
        rsb = sb;
        rinf = (int)min(len, (int64_t)0x7fffffff);
      }
    }
    // row index, first token and length of wave-row k (wave-uniform k)
    auto row_of = [&](int k) {
      if constexpr (kHelp)
        return it.i0 + (int)((uint32_t)__builtin_amdgcn_readlane(rinf, k) >> 24);
      else
        return it.i0 + 2 * wv + 2 * kSimWaves * (k >> 1) + (k & 1);
    };
    auto rinfo = [&](int k, int64_t &sb, int &len) {
      sb = readlane64(rsb, k);
      if constexpr (kHelp) {
        len = __builtin_amdgcn_readlane(rinf, k) & 0xFFFFFF;
        if (len == 0xFFFFFF) {  // a saturated length: read it again
          const int i = row_of(k);
          len = (int)min(clamp64(soffs[i + 1], sb, a.n_src_tok) - sb, (int64_t)0x7fffffff);
        }
      } else {
        len = __builtin_amdgcn_readlane(rinf, k);
      }
    };

    for (int j0 = 0; j0 < m;) {
      if (tid < 64) chunk_end(toffs, j0, m, a.n_tgt_tok, &sh_j1, sh_ends);
      if (tid == 0) sh_nlid = 0;
      for (int s = tid; s < kUcap; s += kSimThreads) uent[s] = make_int2(kEmpty, 0);
      __syncthreads();
      const int j1 = sh_j1;
      const int nj = j1 - j0;
      const int64_t tbase = clamp64(toffs[j0], 0, a.n_tgt_tok);
      const int ntok = min(sh_ends[nj - 1], kTcap);
      // the chunk's tokens, up to kTcap / kSimThreads per thread: all loads in flight at once
      constexpr int kTpt = kTcap / kSimThreads;
      static_assert(kTpt * kSimThreads == kTcap, "every staged token has a thread");
      int32_t xs[kTpt];
#pragma unroll
      for (int u = 0; u < kTpt; u++) {
        const int p = tid + kSimThreads * u;
        xs[u] = p < ntok ? a.tgt_tok[tbase + p] : -1;
      }
      // the chunk's sentences, one per lane of the first wave: local start,
      // length, start in the padded staging (each padded to a multiple of 4
      // with "no id"), by a wave-wide scan
      if (tid < 64) {
        int ostart = 0, blen = 0;
        if (lane < nj) {
          ostart = lane == 0 ? 0 : min(sh_ends[lane - 1], ntok);
          blen = min(max(sh_ends[lane], ostart), ntok) - ostart;
        }
        const int plen = (blen + 3) & ~3;
        int x = plen;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int y = __shfl_up(x, o);
          if (lane >= o) x += y;
        }
        const int pstart = x - plen;
        if (lane < nj) {
          toff_o[lane] = (uint16_t)ostart;
          tlen[lane] = (uint16_t)blen;
          toff[lane] = (uint16_t)pstart;
          for (int q = blen; q < plen; q++) tdoc[pstart + q] = 0xFFFF;
        }
        if (lane == 0) toff_o[nj] = (uint16_t)ntok;
        if (lane == 63) sh_npad = x;
      }
      __syncthreads();
      const int npad = sh_npad;
      // Each token goes into the hash; a key new to the chunk takes the next
      // dense local id (1, 2, ...; one LDS atomic per wave and round, 0 = "no
      // such id", its mask word stays 0).
#pragma unroll
      for (int u = 0; u < kTpt; u++) {
        const int p = tid + kSimThreads * u;
        bool fresh = false;
        int h = 0xFFFF, dst = -1;
        if (p < ntok) {
          int lo = 0;  // sentence holding token p: the last start <= p (starts are non-decreasing)
#pragma unroll
          for (int step = kJcap / 2; step >= 1; step >>= 1)
            if (lo + step < nj && toff_o[lo + step] <= p) lo += step;
          dst = toff[lo] + (p - toff_o[lo]);
          if (xs[u] >= 0) h = u2_insert_fresh(uent, xs[u], fresh);
        }
        const uint64_t nb = __ballot(fresh);
        if (nb) {
          const int lead = __builtin_ctzll(nb);
          int base = 0;
          if (lane == lead) base = atomicAdd(&sh_nlid, __popcll(nb));
          base = __builtin_amdgcn_readlane(base, lead);
          if (fresh) uent[h].y = 1 + base + __popcll(nb & ((1ull << lane) - 1));
        }
        if (dst >= 0) tdoc[dst] = (uint16_t)h;
      }
      __syncthreads();
      const int nlid = sh_nlid + 1;
      for (int q = tid; q < npad; q += kSimThreads) {
        const uint16_t s = tdoc[q];
        tdoc[q] = s == 0xFFFF ? (uint16_t)0 : (uint16_t)uent[s].y;
      }
      __syncthreads();

      // this lane's target sentence and the LDS byte addresses of its mask
      // entries in this wave's array (8 bytes per local id)
      const bool jok = lane < nj;
      const int bl = jok ? tlen[lane] : 0;  // length of target sentence `lane` (this lane's column)
      // When a chunk holds sentences of more than 32 tokens, lanes it leaves
      // over help with the reads: sentence j gets g_j = next_pow2(ceil(b_j /
      // T)) lanes for the smallest T in 4, 8, ..., 32 with sum_j g_j <= 64 (no
      // help if there is none).  Every read then comes from registers (none
      // of the extra id reads of long sentences); the mask reads themselves
      // are as many as before, so chunks of short sentences gain nothing from
      // helpers and get none.  Groups are laid out largest first, so each
      // starts at a multiple of its size; lane L reads one segment of its
      // group's sentence, the group's counts are combined by an xor butterfly
      // and lane j takes them from its group's first lane.
      const int maxb0 = __builtin_amdgcn_readfirstlane(wave_max(bl));
      int gcnt = jok ? 1 : 0, T = 0;
      for (int t = 4; kHelp && maxb0 > kRegTok && t <= kRegTok; t += 4) {
        const int q = (bl + t - 1) / t;
        const int c = jok ? (q <= 1 ? 1 : 1 << (32 - __clz(q - 1))) : 0;
        if (wave_sum(c) <= 64) {
          T = t;
          gcnt = c;
          break;
        }
      }
      // worth it only when the reads saved outweigh the combining (in units
      // of one 8-byte read per lane: register batches of 8 ids, then 5 reads
      // per 4 ids beyond the first 32)
      auto rcost = [](int x) { return 8 * ((min(x, kRegTok) + 7) >> 3) + 5 * ((max(0, x - kRegTok) + 3) >> 2); };
      if (T > 0) {
        const int mg = __builtin_amdgcn_readfirstlane(wave_max(gcnt));
        if (rcost(T) + 4 + 2 * (31 - __clz(mg)) >= rcost(maxb0)) T = 0;
      }
      if (T == 0) gcnt = jok ? 1 : 0;
      const bool helped = T > 0;  // wave-uniform
      int gbase = lane;           // first lane of sentence `lane`'s group
      int rl = bl, rgs = 1;       // this lane's read length and its group's size
      const uint16_t *rp = tdoc + (jok ? toff[lane] : 0);
      int maxgs = 1;
      if (helped) {
        int off = 0;
        gbase = 0;
        for (int sz = 64; sz >= 1; sz >>= 1) {
          const uint64_t mk = __ballot(gcnt == sz);
          if (gcnt == sz) gbase = off + sz * __popcll(mk & ((1ull << lane) - 1));
          off += sz * __popcll(mk);
        }
        sh_own[wv][lane] = 0xFF;
        wave_sync();
        for (int e = 0; e < gcnt; e++) sh_own[wv][gbase + e] = (uint8_t)lane;
        wave_sync();
        const int js = sh_own[wv][lane];
        const int jsc = js == 0xFF ? 0 : js;
        const int gsz = __shfl(gcnt, jsc), gb = __shfl(gbase, jsc);
        rl = 0;
        if (js != 0xFF) {
          rgs = gsz;
          const int b = tlen[js];
          const int seg = ((b + rgs - 1) / rgs + 3) & ~3;  // a multiple of 4: 8-byte aligned id reads
          const int ts = min(b, (lane - gb) * seg);
          rl = min(b, ts + seg) - ts;
          rp = tdoc + toff[js] + ts;
        }
        maxgs = __builtin_amdgcn_readfirstlane(wave_max(gcnt));
        wave_sync();
      }
      const uint16_t *const tp = rp;
      const uint32_t wbase = mw_lds + (uint32_t)wv * (kTcap + 4) * 8u;
      uint32_t ad[kRegTok];
#pragma unroll
      for (int k = 0; k < kRegTok; k++) {
        ad[k] = wbase + (k < rl ? (uint32_t)tp[k] * 8u : 0u);
        asm volatile("" : "+v"(ad[k]));  // keep the whole address in the register (no add per read)
      }
      const int maxb = __builtin_amdgcn_readfirstlane(wave_max(rl));
      const uint32_t grp = (uint32_t)gbase | ((uint32_t)rgs << 8);  // both in one register
      // Combine a group's partial results (two masks OR-ed, one packed sum
      // added) with an xor-style butterfly; afterwards every lane of a group
      // holds the group's totals.
      auto butterfly = [&](uint32_t &o0, uint32_t &o1, uint32_t &sp, uint32_t *sq) {
        uint32_t sq0 = sq ? *sq : 0u;
        if (maxgs > 1) {
          const uint32_t a0 = dpp_mov<0xB1>(o0), a1 = dpp_mov<0xB1>(o1), b = dpp_mov<0xB1>(sp);
          const uint32_t c = sq ? dpp_mov<0xB1>(sq0) : 0u;
          if ((grp >> 8) > 1u) o0 |= a0, o1 |= a1, sp += b, sq0 += c;
        }
        if (maxgs > 2) {
          const uint32_t a0 = dpp_mov<0x4E>(o0), a1 = dpp_mov<0x4E>(o1), b = dpp_mov<0x4E>(sp);
          const uint32_t c = sq ? dpp_mov<0x4E>(sq0) : 0u;
          if ((grp >> 8) > 2u) o0 |= a0, o1 |= a1, sp += b, sq0 += c;
        }
        if (maxgs > 4) {
          const uint32_t a0 = dpp_mov<0x141>(o0), a1 = dpp_mov<0x141>(o1), b = dpp_mov<0x141>(sp);
          const uint32_t c = sq ? dpp_mov<0x141>(sq0) : 0u;
          if ((grp >> 8) > 4u) o0 |= a0, o1 |= a1, sp += b, sq0 += c;
        }
        if (maxgs > 8) {
          const uint32_t a0 = dpp_mov<0x140>(o0), a1 = dpp_mov<0x140>(o1), b = dpp_mov<0x140>(sp);
          const uint32_t c = sq ? dpp_mov<0x140>(sq0) : 0u;
          if ((grp >> 8) > 8u) o0 |= a0, o1 |= a1, sp += b, sq0 += c;
        }
        for (int dd = 16; dd < maxgs; dd <<= 1) {
          const uint32_t a0 = __shfl_xor(o0, dd), a1 = __shfl_xor(o1, dd), b = __shfl_xor(sp, dd);
          const uint32_t c = sq ? (uint32_t)__shfl_xor((int)sq0, dd) : 0u;
          if ((uint32_t)dd < (grp >> 8)) o0 |= a0, o1 |= a1, sp += b, sq0 += c;
        }
        if (sq) *sq = sq0;
      };
      // two-row step: position masks of both rows (hit bit 31) and hit counts
      // -> m_s and m_t of both rows at lane = sentence
      auto counts2 = [&](uint32_t o0, uint32_t o1, uint32_t t0, uint32_t t1, int &ms0, int &ms1, int &mt0, int &mt1) {
        if (!helped) {
          ms0 = __popc(o0 & ~kHitBit), ms1 = __popc(o1 & ~kHitBit), mt0 = (int)t0, mt1 = (int)t1;
          return;
        }
        uint32_t sp = t0 | (t1 << 16);  // each count <= kTcap < 2^11
        butterfly(o0, o1, sp, nullptr);
        const uint32_t pk = __popc(o0 & ~kHitBit) | (__popc(o1 & ~kHitBit) << 5) | ((sp & 0x7FFu) << 10) | (((sp >> 16) & 0x7FFu) << 21);
        const uint32_t g = (uint32_t)__shfl((int)pk, (int)(grp & 0xFFu));
        ms0 = g & 31u, ms1 = (g >> 5) & 31u, mt0 = (g >> 10) & 0x7FFu, mt1 = g >> 21;
      };
      // four-row step: fields of rows 0, 1 in o0 and 2, 3 in o1 (15 position
      // bits and the hit bit each); hit counts of rows 0, 1 in the 16-bit
      // halves of h0, of rows 2, 3 in h1
      auto counts4 = [&](uint32_t o0, uint32_t o1, uint32_t h0, uint32_t h1, int *ms, int *mt) {
        if (helped) {
          butterfly(o0, o1, h0, &h1);
          const uint32_t pa = h0 | ((uint32_t)__popc(o0 & 0x7FFFu) << 11) | ((uint32_t)__popc(o0 & 0x7FFF0000u) << 27);
          const uint32_t pb = h1 | ((uint32_t)__popc(o1 & 0x7FFFu) << 11) | ((uint32_t)__popc(o1 & 0x7FFF0000u) << 27);
          const uint32_t ga = (uint32_t)__shfl((int)pa, (int)(grp & 0xFFu));
          const uint32_t gb = (uint32_t)__shfl((int)pb, (int)(grp & 0xFFu));
          ms[0] = (ga >> 11) & 15u, ms[1] = ga >> 27, mt[0] = ga & 0x7FFu, mt[1] = (ga >> 16) & 0x7FFu;
          ms[2] = (gb >> 11) & 15u, ms[3] = gb >> 27, mt[2] = gb & 0x7FFu, mt[3] = (gb >> 16) & 0x7FFu;
          return;
        }
        ms[0] = __popc(o0 & 0x7FFFu), ms[1] = __popc(o0 & 0x7FFF0000u);
        ms[2] = __popc(o1 & 0x7FFFu), ms[3] = __popc(o1 & 0x7FFF0000u);
        mt[0] = h0 & 0xFFFFu, mt[1] = h0 >> 16, mt[2] = h1 & 0xFFFFu, mt[3] = h1 >> 16;
      };
      // one-row pass: a 64-bit position mask (hit bit 63) and the hit count
      auto counts1 = [&](uint32_t o0, uint32_t o1, uint32_t t, int &ms, int &mt) {
        if (!helped) {
          ms = __popc(o0) + __popc(o1 & ~kHitBit), mt = (int)t;
          return;
        }
        butterfly(o0, o1, t, nullptr);
        const uint32_t pk = (__popc(o0) + __popc(o1 & ~kHitBit)) | (t << 6);
        const uint32_t g = (uint32_t)__shfl((int)pk, (int)(grp & 0xFFu));
        ms = g & 63u, mt = g >> 6;
      };
      const int ng = (min(maxb, kRegTok) + 3) >> 2;
      const int nq4 = (nlid + 1) >> 1;  // 16-byte stores covering the chunk's entries

      // Score of cell (i, j0 + lane) from its counts, and its offset in the
      // pair's score block (-1: no cell).  The two-row steps store their
      // scores two steps later (two sets of pending scores, one per call site
      // of the unrolled loop), so the table reads are not waited for while
      // the next rows are worked on.
      float *const Sb = a.S + d.s_off;
      // A step's two rows i, i + 1 lie in one strip, where cell (i + 1, c - 1)
      // follows cell (i, c): lane c stores both as one 8-byte store (strips of
      // an even row count; the pair's block starts 16-byte aligned).
      struct Pend {
        int o0 = -1, oB = -1;  // o0: cell (i, c), paired with (i + 1, c - 1); oB: (i + 1, c) alone
        float v0 = 0.0f, vl = 0.0f, vB = 0.0f;
        bool paired = false;
      };
      auto flush = [&](Pend &q) {
        if (q.o0 >= 0) {
          if (q.paired)
            *reinterpret_cast<float2 *>(Sb + q.o0) = make_float2(q.v0, q.vl);
          else
            Sb[q.o0] = q.v0;
        }
        if (q.oB >= 0) Sb[q.oB] = q.vB;
      };
      auto score_cell = [&](int i, int ai, uint32_t ms, uint32_t mt, int &off) -> float {
        // the table read is issued by every lane (clamped index), so no branch
        // hides it from the wait-count bookkeeping
        const int ca = min(ai, kTabLen - 1), cb = min(bl, kTabLen - 1);
        const int cs = min((int)ms, kTabLen - 1), ct = min((int)mt, kTabLen - 1);
        float sv = a.table[tab_index(ca, cb, cs, ct)];
        off = -1;
        if (!jok) return 0.0f;
        if (ai >= kTabLen || bl >= kTabLen) sv = score_direct(a.w0, a.w1, a.w2, a.w3, (int)ms, ai, (int)mt, bl);
        off = (int)score_pos(i, j0 + lane, n, m);
        if (a.ms_out) {
          const int64_t cell = d.rm_off + (int64_t)i * m + j0 + lane;
          a.ms_out[cell] = (int)ms;
          a.mt_out[cell] = (int)mt;
        }
        return sv;
      };

      // One row at a time (sentences of more than 31 tokens): lane q holds
      // source position q < 64.  A mask entry is one 64-bit word here: bits
      // 0-62 are positions, bit 63 the hit bit, so one pass covers 63
      // positions (longer sentences take further passes, position bits only).
      auto single_row = [&](const int k) {
        const int i = row_of(k);
        int64_t sb;
        int ai;
        rinfo(k, sb, ai);
        const int4 cur = lane < ai ? a.trans[sb + lane] : make_int4(-1, -1, -1, -1);
        unsigned long long *Mq = reinterpret_cast<unsigned long long *>(Mx);
        constexpr int kPass = 63;
        uint32_t ms_acc = 0, mt_acc = 0;
        const int npass = ai <= kPass ? 1 : (ai + kPass - 1) / kPass;
        for (int c = 0; c < npass; c++) {
          const int qlo = c == 0 ? 0 : kPass * c;
          const int qhi = c == 0 ? ai : min(ai, kPass * c + kPass);
          for (int q = qlo + lane; q < qhi; q += 64) {
            const int4 t4 = (c == 0 && q < 64) ? cur : a.trans[sb + q];  // cur holds position `lane`
            const int rel = q - kPass * c;
            const unsigned long long bits =
                (c == 0 ? (1ull << 63) : 0ull) | (rel >= 0 && rel < kPass ? (1ull << rel) : 0ull);
            if (t4.x == -2) {
              for (int e = 0; e < t4.z; e++) {
                const int l = u2_lid(uent, a.lex.vals[t4.y + e]);
                if (l) atomicOr(&Mq[l], bits);
              }
            } else {
              const int4 lid = u2_lid4(uent, t4);
              const int l0 = lid.x, l1 = lid.y, l2 = lid.z, l3 = lid.w;
              if (l0) atomicOr(&Mq[l0], bits);
              if (l1) atomicOr(&Mq[l1], bits);
              if (l2) atomicOr(&Mq[l2], bits);
              if (l3) atomicOr(&Mq[l3], bits);
            }
          }
          wave_sync();
          uint32_t acc0 = 0, acc1 = 0, mt = 0;
#pragma unroll
          for (int g = 0; g < kRegTok / 8; g++) {
            if (2 * g < ng) {
              uint2 w[8];
#pragma unroll
              for (int u = 0; u < 8; u++) w[u] = lds_u2_at(ad[8 * g + u]);
#pragma unroll
              for (int u = 0; u < 8; u += 4) {
                mt += ((w[u].y >> 31) + (w[u + 1].y >> 31)) + ((w[u + 2].y >> 31) + (w[u + 3].y >> 31));
                acc0 |= (w[u].x | w[u + 1].x) | (w[u + 2].x | w[u + 3].x);
                acc1 |= (w[u].y | w[u + 1].y) | (w[u + 2].y | w[u + 3].y);
              }
            }
          }
          // sentences beyond 32 tokens: the rest straight from LDS, four ids per
          // read (sentences are padded to a multiple of 4 with id 0)
          for (int k2 = kRegTok; k2 < maxb; k2 += 4) {
            if (k2 < bl) {  // only chunks without helpers get here (rl == bl)
              const uint2 ids = *reinterpret_cast<const uint2 *>(tp + k2);
              const uint2 w0 = *reinterpret_cast<const uint2 *>(Mx + 2 * (ids.x & 0xFFFFu));
              const uint2 w1 = *reinterpret_cast<const uint2 *>(Mx + 2 * (ids.x >> 16));
              const uint2 w2 = *reinterpret_cast<const uint2 *>(Mx + 2 * (ids.y & 0xFFFFu));
              const uint2 w3 = *reinterpret_cast<const uint2 *>(Mx + 2 * (ids.y >> 16));
              mt += ((w0.y >> 31) + (w1.y >> 31)) + ((w2.y >> 31) + (w3.y >> 31));
              acc0 |= (w0.x | w1.x) | (w2.x | w3.x);
              acc1 |= (w0.y | w1.y) | (w2.y | w3.y);
            }
          }
          int msp, mtp;
          counts1(acc0, acc1, mt, msp, mtp);
          ms_acc += msp;
          if (c == 0) mt_acc = mtp;
          wave_sync();
          for (int k2 = lane; k2 < nq4; k2 += 64) reinterpret_cast<uint4 *>(Mx)[k2] = make_uint4(0, 0, 0, 0);
          wave_sync();
        }
        int off;
        const float sv = score_cell(i, ai, ms_acc, mt_acc, off);
        if (off >= 0) Sb[off] = sv;
      };

      // Two rows at a time (both of at most 31 tokens): lanes 0-31 hold the
      // positions of row k, lanes 32-63 those of row k + 1; row k marks the
      // first word of each entry and row k + 1 the second, so one 8-byte read
      // per target token serves both rows.  The translations of the next two
      // rows are fetched while these are worked on.
      // two-row steps take wave-rows k and k + 1 of [nQ, nP2)
      const int nP2 = nQ + nP;
      auto fetch2 = [&](int k) -> int4 {
        int64_t b0 = 0, b1 = 0;
        int n0 = 0, n1 = 0;
        if constexpr (kHelp) {
          if (k < nP2) rinfo(k, b0, n0);
          if (k + 1 < nP2) rinfo(k + 1, b1, n1);
        } else {
          b0 = readlane64(rsb, min(k, 63)), b1 = readlane64(rsb, min(k + 1, 63));
          n0 = k < nrows ? __builtin_amdgcn_readlane(rinf, min(k, 63)) : 0;
          n1 = k + 1 < nrows ? __builtin_amdgcn_readlane(rinf, min(k + 1, 63)) : 0;
        }
        const int q = lane & 31, len = lane < 32 ? n0 : n1;
        const bool ok = q < len && len <= kPosBits;
        // every lane reads (a valid token's record: clamped), then keeps it or not
        const int64_t at = ok ? (lane < 32 ? b0 : b1) + q : 0;
        const int4 r = a.trans[at];
        return ok ? r : make_int4(-1, -1, -1, -1);
      };
      auto pair_rows = [&](const int k, const int4 cur, Pend &pend) {
        const bool has1 = k + 1 < nP2;
        int ai0, ai1 = 0;
        if constexpr (kHelp) {
          int64_t sbx;
          rinfo(k, sbx, ai0);
          if (has1) rinfo(k + 1, sbx, ai1);
        } else {
          ai0 = __builtin_amdgcn_readlane(rinf, k);
          ai1 = has1 ? __builtin_amdgcn_readlane(rinf, k + 1) : 0;
        }
        if constexpr (!kHelp) {  // kernel 2's row classes leave no long row here
          if (ai0 > kPosBits || ai1 > kPosBits) {
            single_row(k);
            if (has1) single_row(k + 1);
            return;
          }
        }
        const int half = lane >> 5, q = lane & 31;
        const int aih = half ? ai1 : ai0;
        const bool mine = q < aih;
        const bool far = cur.x == -2;  // more than four translations
        const int4 lid = u2_lid4(uent, far ? make_int4(-1, -1, -1, -1) : cur);
        const int l0 = lid.x, l1 = lid.y, l2 = lid.z, l3 = lid.w;
        uint32_t *Mh = Mx + half;  // this half's word of entry l: Mh[2 l]
        const uint32_t bits = kHitBit | (1u << q);
        if (mine) {
          if (far) {
            for (int e = 0; e < cur.z; e++) {
              const int l = u2_lid(uent, a.lex.vals[cur.y + e]);
              if (l) atomicOr(&Mh[2 * l], bits);
            }
          } else {
            if (l0) atomicOr(&Mh[2 * l0], bits);
            if (l1) atomicOr(&Mh[2 * l1], bits);
            if (l2) atomicOr(&Mh[2 * l2], bits);
            if (l3) atomicOr(&Mh[2 * l3], bits);
          }
        }
        wave_sync();
        // eight entries per batch (entries past a sentence's end are entry 0, always zero)
        uint32_t acc0 = 0, mt0 = 0, acc1 = 0, mt1 = 0;
#pragma unroll
        for (int g = 0; g < kRegTok / 8; g++) {
          if (2 * g < ng) {
            uint2 w[8];
#pragma unroll
            for (int u = 0; u < 8; u++) w[u] = lds_u2_at(ad[8 * g + u]);
#pragma unroll
            for (int u = 0; u < 8; u += 4) {
              mt0 += ((w[u].x >> 31) + (w[u + 1].x >> 31)) + ((w[u + 2].x >> 31) + (w[u + 3].x >> 31));
              acc0 |= (w[u].x | w[u + 1].x) | (w[u + 2].x | w[u + 3].x);
              mt1 += ((w[u].y >> 31) + (w[u + 1].y >> 31)) + ((w[u + 2].y >> 31) + (w[u + 3].y >> 31));
              acc1 |= (w[u].y | w[u + 1].y) | (w[u + 2].y | w[u + 3].y);
            }
          }
        }
        for (int k2 = kRegTok; k2 < maxb; k2 += 4) {  // beyond 32 tokens, four ids per read
          if (k2 < bl) {  // only chunks without helpers get here (rl == bl)
            const uint2 ids = *reinterpret_cast<const uint2 *>(tp + k2);
            const uint2 w0 = *reinterpret_cast<const uint2 *>(Mx + 2 * (ids.x & 0xFFFFu));
            const uint2 w1 = *reinterpret_cast<const uint2 *>(Mx + 2 * (ids.x >> 16));
            const uint2 w2 = *reinterpret_cast<const uint2 *>(Mx + 2 * (ids.y & 0xFFFFu));
            const uint2 w3 = *reinterpret_cast<const uint2 *>(Mx + 2 * (ids.y >> 16));
            mt0 += ((w0.x >> 31) + (w1.x >> 31)) + ((w2.x >> 31) + (w3.x >> 31));
            acc0 |= (w0.x | w1.x) | (w2.x | w3.x);
            mt1 += ((w0.y >> 31) + (w1.y >> 31)) + ((w2.y >> 31) + (w3.y >> 31));
            acc1 |= (w0.y | w1.y) | (w2.y | w3.y);
          }
        }
        int ms0, ms1, mc0, mc1;
        counts2(acc0, acc1, mt0, mt1, ms0, ms1, mc0, mc1);
        wave_sync();
        if (mine) {
          if (far) {
            for (int e = 0; e < cur.z; e++) {
              const int l = u2_lid(uent, a.lex.vals[cur.y + e]);
              if (l) Mh[2 * l] = 0;
            }
          } else {
            if (l0) Mh[2 * l0] = 0;
            if (l1) Mh[2 * l1] = 0;
            if (l2) Mh[2 * l2] = 0;
            if (l3) Mh[2 * l3] = 0;
          }
        }
        wave_sync();
        const int i = row_of(k), i1 = has1 ? row_of(k + 1) : -1;
        int off0, off1 = -1;
        const float sv0 = score_cell(i, ai0, ms0, mc0, off0);
        float sv1 = 0.0f;
        if (has1) sv1 = score_cell(i1, ai1, ms1, mc1, off1);
        // rows i and i + 1 (i even) of a strip with an even row count: 8-byte
        // stores (kernel 1's two rows always are i and i + 1 with i even)
        const bool adjacent = kHelp ? (i1 == i + 1 && (i & 1) == 0) : has1;
        const bool pairable = adjacent && ((min(64, n - ((i >> 6) << 6)) & 1) == 0);
        const float left_v = shift_up_one_lane(sv1);  // lane c: cell (i + 1, c - 1)
        const int left_o = __shfl_up(off1, 1);
        const bool paired = pairable && lane >= 1 && off0 >= 0 && left_o >= 0;
        const bool right_pairs = __shfl_down(paired ? 1 : 0, 1) != 0 && lane < 63;
        flush(pend);  // this call site's scores of two steps ago
        pend.o0 = off0;
        pend.v0 = sv0;
        pend.vl = left_v;
        pend.paired = paired;
        pend.oB = (off1 >= 0 && !right_pairs) ? off1 : -1;
        pend.vB = sv1;
      };
      if constexpr (kHelp) {
        // Four rows at a time (all of at most 15 tokens): lanes 16 r + q hold
        // position q of row r, and row r marks its 16-bit field of the entry
        // (half r & 1 of word r >> 1): position bits 0-14, hit bit 15.
        const int cq = (nQ + 3) >> 2;  // four-row units: wave-rows 4 t ..
        auto fetch4 = [&](int t) -> int4 {
          const int r = lane >> 4, q = lane & 15;
          int64_t sbr = 0;
          int len = 0;
  #pragma unroll
          for (int rr = 0; rr < 4; rr++) {
            if (t < cq && 4 * t + rr < nQ) {
              int64_t b;
              int l;
              rinfo(4 * t + rr, b, l);
              if (r == rr) sbr = b, len = l;
            }
          }
          const bool ok = q < len && len <= kQuadBits;
          const int64_t at = ok ? sbr + q : 0;
          const int4 rec = a.trans[at];
          return ok ? rec : make_int4(-1, -1, -1, -1);
        };
        struct PendQ {
          int o[4] = {-1, -1, -1, -1};
          float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        };
        auto flushQ = [&](PendQ &q) {
  #pragma unroll
          for (int rr = 0; rr < 4; rr++)
            if (q.o[rr] >= 0) Sb[q.o[rr]] = q.v[rr];
        };
        auto quad_rows = [&](const int t, const int4 cur, PendQ &pend) {
          const int r = lane >> 4, q = lane & 15;
          const bool far = cur.x == -2;  // more than four translations
          const int4 lid = u2_lid4(uent, far ? make_int4(-1, -1, -1, -1) : cur);
          const int l0 = lid.x, l1 = lid.y, l2 = lid.z, l3 = lid.w;
          uint32_t *Mh = Mx + (r >> 1);  // this row's word of entry l: Mh[2 l]
          const uint32_t bits = ((1u << kQuadBits) | (1u << q)) << (16 * (r & 1));
          if (far) {
            for (int e = 0; e < cur.z; e++) {
              const int l = u2_lid(uent, a.lex.vals[cur.y + e]);
              if (l) atomicOr(&Mh[2 * l], bits);
            }
          } else {
            if (l0) atomicOr(&Mh[2 * l0], bits);
            if (l1) atomicOr(&Mh[2 * l1], bits);
            if (l2) atomicOr(&Mh[2 * l2], bits);
            if (l3) atomicOr(&Mh[2 * l3], bits);
          }
          wave_sync();
          uint32_t ox = 0, oy = 0, hx = 0, hy = 0;
  #pragma unroll
          for (int g = 0; g < kRegTok / 8; g++) {
            if (2 * g < ng) {
              uint2 w[8];
  #pragma unroll
              for (int u = 0; u < 8; u++) w[u] = lds_u2_at(ad[8 * g + u]);
  #pragma unroll
              for (int u = 0; u < 8; u += 4) {
                hx += ((w[u].x >> 15) & 0x10001u) + ((w[u + 1].x >> 15) & 0x10001u) + ((w[u + 2].x >> 15) & 0x10001u) +
                      ((w[u + 3].x >> 15) & 0x10001u);
                hy += ((w[u].y >> 15) & 0x10001u) + ((w[u + 1].y >> 15) & 0x10001u) + ((w[u + 2].y >> 15) & 0x10001u) +
                      ((w[u + 3].y >> 15) & 0x10001u);
                ox |= (w[u].x | w[u + 1].x) | (w[u + 2].x | w[u + 3].x);
                oy |= (w[u].y | w[u + 1].y) | (w[u + 2].y | w[u + 3].y);
              }
            }
          }
          for (int k2 = kRegTok; k2 < maxb; k2 += 4) {  // beyond 32 tokens, four ids per read
            if (k2 < bl) {  // only chunks without helpers get here (rl == bl)
              const uint2 ids = *reinterpret_cast<const uint2 *>(tp + k2);
              const uint2 w0 = *reinterpret_cast<const uint2 *>(Mx + 2 * (ids.x & 0xFFFFu));
              const uint2 w1 = *reinterpret_cast<const uint2 *>(Mx + 2 * (ids.x >> 16));
              const uint2 w2 = *reinterpret_cast<const uint2 *>(Mx + 2 * (ids.y & 0xFFFFu));
              const uint2 w3 = *reinterpret_cast<const uint2 *>(Mx + 2 * (ids.y >> 16));
              hx += ((w0.x >> 15) & 0x10001u) + ((w1.x >> 15) & 0x10001u) + ((w2.x >> 15) & 0x10001u) + ((w3.x >> 15) & 0x10001u);
              hy += ((w0.y >> 15) & 0x10001u) + ((w1.y >> 15) & 0x10001u) + ((w2.y >> 15) & 0x10001u) + ((w3.y >> 15) & 0x10001u);
              ox |= (w0.x | w1.x) | (w2.x | w3.x);
              oy |= (w0.y | w1.y) | (w2.y | w3.y);
            }
          }
          int ms[4], mt[4];
          counts4(ox, oy, hx, hy, ms, mt);
          wave_sync();
          if (far) {
            for (int e = 0; e < cur.z; e++) {
              const int l = u2_lid(uent, a.lex.vals[cur.y + e]);
              if (l) Mh[2 * l] = 0;
            }
          } else {
            if (l0) Mh[2 * l0] = 0;
            if (l1) Mh[2 * l1] = 0;
            if (l2) Mh[2 * l2] = 0;
            if (l3) Mh[2 * l3] = 0;
          }
          wave_sync();
          flushQ(pend);  // this call site's scores of two steps ago
  #pragma unroll
          for (int rr = 0; rr < 4; rr++) {
            pend.o[rr] = -1;
            if (4 * t + rr < nQ) {
              int64_t sbx;
              int ai;
              rinfo(4 * t + rr, sbx, ai);
              pend.v[rr] = score_cell(row_of(4 * t + rr), ai, ms[rr], mt[rr], pend.o[rr]);
            }
          }
        };

        // One call site per step kind (code size): the prefetched records and
        // the two pending sets trade places after every step.
        {  // four-row units
          int4 fa = fetch4(0);
          PendQ pa, pb;
          for (int t = 0; t < cq; t++) {
            const int4 fb = fetch4(t + 1);
            quad_rows(t, fa, pa);
            fa = fb;
            const PendQ px = pa;
            pa = pb;
            pb = px;
          }
          flushQ(pa);
          flushQ(pb);
        }
        {  // two-row units
          int4 fa = fetch2(nQ);
          Pend qa, qb;
          for (int k = nQ; k < nP2; k += 2) {
            const int4 fb = fetch2(k + 2);
            pair_rows(k, fa, qa);
            fa = fb;
            const Pend qx = qa;
            qa = qb;
            qb = qx;
          }
          flush(qa);
          flush(qb);
        }
        for (int t = 0; t < nL; t++) single_row(nQ + nP + t);  // one-row units
      } else {
        int4 bufA = fetch2(0), bufB;
        Pend qa, qb;
        for (int k = 0; k < nrows; k += 4) {
          bufB = fetch2(k + 2);
          pair_rows(k, bufA, qa);
          if (k + 2 >= nrows) break;
          bufA = fetch2(k + 4);
          pair_rows(k + 2, bufB, qb);
        }
        flush(qa);
        flush(qb);
      }
      __syncthreads();
      j0 = j1;
    }
  }
}

// The tile kernel computes the same counts as sim_kernel with far fewer
// instructions per cell.  A work item is (pair, source rows [i0, i1)) with i0
// a multiple of 128; wave w owns the 64-row strip starting at i0 + 64 w.
// Target sentences are taken in chunks of at most 64 sentences / kTcap
// tokens, staged in LDS with dense local ids as in sim_kernel, plus
//   D[id] = set of the chunk's target sentences holding id (64-bit word).
// For its strip a wave builds
//   B[id] = set of the strip's source sentences whose X_i holds id,
// and counts with bit-sliced counters (plane b holds bit b of 64 counts):
//   source pass, lane = source sentence i: for each token q, the OR of
//     D[id] over the token's translations is the set of target sentences j
//     that meet T(s_i[q]); adding it counts m_s(i, .) for all 64 j at once;
//   target pass, lane = target sentence j: for each token p, B[id(t_j[p])]
//     is the set of source sentences i with t_j[p] in X_i; adding it counts
//     m_t(., j) for all 64 i at once.
// A 64 x 64 bit-matrix transpose through lane shuffles turns the m_s planes
// around so that lane j holds both counts of its 64 cells, scores them and
// stores them.
constexpr int kTileWaves = 2;
constexpr int kTileThreads = 64 * kTileWaves;
constexpr int kFastPlanes = 6;   // counts <= 63 (sentences of at most 63 tokens)
constexpr int kWidePlanes = 11;  // counts <= 2047

template <int NW>
__device__ __forceinline__ int block_excl_sum(int v, int *sh, int *total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wv] = x;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NW; w++) {
    const int s = sh[w];
    base += (w < wv) ? s : 0;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

// add a 64-bit set (one bit per counter) into NPL bit-sliced planes
template <int NPL>
__device__ __forceinline__ void bs_add(uint32_t (&lo)[NPL], uint32_t (&hi)[NPL], uint32_t xl, uint32_t xh) {
#pragma unroll
  for (int b = 0; b < NPL; b++) {
    const uint32_t tl = lo[b] & xl, th = hi[b] & xh;
    lo[b] ^= xl;
    hi[b] ^= xh;
    xl = tl;
    xh = th;
  }
}

// transpose a 64 x 64 bit matrix held one row per lane (bit c of lane l's
// word = M[l][c]); afterwards lane c holds column c (bit l = M[l][c])
__device__ __forceinline__ void transpose64(uint32_t &lo, uint32_t &hi, int lane) {
  {
    const uint32_t ylo = __shfl_xor(lo, 32), yhi = __shfl_xor(hi, 32);
    const bool up = (lane & 32) != 0;
    lo = up ? yhi : lo;
    hi = up ? hi : ylo;
  }
#pragma unroll
  for (int s = 16; s >= 1; s >>= 1) {
    const uint32_t m = s == 16 ? 0x0000FFFFu : s == 8 ? 0x00FF00FFu : s == 4 ? 0x0F0F0F0Fu : s == 2 ? 0x33333333u : 0x55555555u;
    const uint32_t ylo = __shfl_xor(lo, s), yhi = __shfl_xor(hi, s);
    const bool up = (lane & s) != 0;
    const uint32_t alo = (lo & m) | ((ylo & m) << s), ahi = (hi & m) | ((yhi & m) << s);
    const uint32_t blo = (lo & ~m) | ((ylo & ~m) >> s), bhi = (hi & ~m) | ((yhi & ~m) >> s);
    lo = up ? blo : alo;
    hi = up ? bhi : ahi;
  }
}

template <int NPL>
__device__ __forceinline__ uint32_t bs_get(const uint32_t (&lo)[NPL], const uint32_t (&hi)[NPL], int l) {
  uint32_t v = 0;
#pragma unroll
  for (int b = 0; b < NPL; b++) v |= ((l < 32 ? lo[b] >> l : hi[b] >> (l - 32)) & 1u) << b;
  return v;
}

struct TileCtx {
  const int32_t *ukey;
  const uint16_t *ulid;
  const uint64_t *D;
  uint64_t *B;
  const uint16_t *tp;  // this lane's staged target ids
  int bl;              // this lane's target sentence length
  bool jok;
  int nj, j0, nlid;
};

// One strip x chunk tile: counts and scores of rows [r0, r0 + R) against the
// chunk's target sentences.
template <int NPL>
__device__ __forceinline__ void tile_work(const SimArgs &a, const PairDesc &d, const int64_t *soffs, int r0, int R,
                                          const TileCtx &t, int lane, int *al_s) {
  uint64_t *B = t.B;
  // clear B
  for (int k = lane; k < t.nlid; k += 64) B[k] = 0;
  wave_sync();

  // ---- source pass: lane = source sentence r0 + lane
  const bool iok = lane < R;
  int64_t sb = 0;
  int al = 0;
  if (iok) {
    sb = clamp64(soffs[r0 + lane], 0, a.n_src_tok);
    const int64_t se = clamp64(soffs[r0 + lane + 1], sb, a.n_src_tok);
    al = (int)min<int64_t>(se - sb, 0x7fffffff);
  }
  const int maxa = wave_max(al);
  uint32_t sl[NPL], sh[NPL];
#pragma unroll
  for (int b = 0; b < NPL; b++) sl[b] = sh[b] = 0;
  const uint64_t mybit = 1ull << lane;
  int4 nxt = al > 0 ? a.trans[sb] : make_int4(-1, -1, -1, -1);
  for (int q = 0; q < maxa; q++) {
    const int4 t4 = nxt;
    nxt = q + 1 < al ? a.trans[sb + q + 1] : make_int4(-1, -1, -1, -1);
    uint64_t C = 0;
    if (q < al) {
      if (t4.x == -2) {
        for (int e = 0; e < t4.z; e++) {
          const int s = u_find(t.ukey, a.lex.vals[t4.y + e]);
          if (s >= 0) {
            const int id = t.ulid[s];
            atomicOr(reinterpret_cast<unsigned long long *>(&B[id]), (unsigned long long)mybit);
            C |= t.D[id];
          }
        }
      } else {
        const int s0 = u_find(t.ukey, t4.x), s1 = u_find(t.ukey, t4.y), s2 = u_find(t.ukey, t4.z),
                  s3 = u_find(t.ukey, t4.w);
        const int id0 = s0 >= 0 ? t.ulid[s0] : 0, id1 = s1 >= 0 ? t.ulid[s1] : 0;
        const int id2 = s2 >= 0 ? t.ulid[s2] : 0, id3 = s3 >= 0 ? t.ulid[s3] : 0;
        if (id0) atomicOr(reinterpret_cast<unsigned long long *>(&B[id0]), (unsigned long long)mybit);
        if (id1) atomicOr(reinterpret_cast<unsigned long long *>(&B[id1]), (unsigned long long)mybit);
        if (id2) atomicOr(reinterpret_cast<unsigned long long *>(&B[id2]), (unsigned long long)mybit);
        if (id3) atomicOr(reinterpret_cast<unsigned long long *>(&B[id3]), (unsigned long long)mybit);
        C = (t.D[id0] | t.D[id1]) | (t.D[id2] | t.D[id3]);  // D[0] = 0
      }
    }
    bs_add<NPL>(sl, sh, (uint32_t)C, (uint32_t)(C >> 32));
  }
  wave_sync();

  // ---- target pass: lane = target sentence j0 + lane
  uint32_t tl[NPL], th[NPL];
#pragma unroll
  for (int b = 0; b < NPL; b++) tl[b] = th[b] = 0;
  const int maxb = wave_max(t.bl);
  for (int k = 0; k < maxb; k += 4) {
    uint64_t x0 = 0, x1 = 0, x2 = 0, x3 = 0;
    if (k < t.bl) {  // ids are padded to a multiple of 4 with id 0 (B[0] = 0)
      const uint2 ids = *reinterpret_cast<const uint2 *>(t.tp + k);
      x0 = B[ids.x & 0xFFFFu];
      x1 = B[ids.x >> 16];
      x2 = B[ids.y & 0xFFFFu];
      x3 = B[ids.y >> 16];
    }
    bs_add<NPL>(tl, th, (uint32_t)x0, (uint32_t)(x0 >> 32));
    bs_add<NPL>(tl, th, (uint32_t)x1, (uint32_t)(x1 >> 32));
    bs_add<NPL>(tl, th, (uint32_t)x2, (uint32_t)(x2 >> 32));
    bs_add<NPL>(tl, th, (uint32_t)x3, (uint32_t)(x3 >> 32));
  }

  // ---- bring m_s(i, j) to lane j
#pragma unroll
  for (int b = 0; b < NPL; b++) transpose64(sl[b], sh[b], lane);

  // ---- score the 64 cells of lane j: rows r0 .. r0 + R - 1
  al_s[lane] = al;  // source lengths, read back with a uniform index
  wave_sync();
  const int n = d.n, m = d.m;
  const int c = t.j0 + lane;
  if (NPL == kFastPlanes) {
    // Cells l0 + 8k (k = 0..3) of a 32-row half at once: one shift and mask
    // per plane gathers their bits into four bytes.
    float *strip = a.S + d.s_off + (int64_t)(r0 >> 6) * (m + 63) * 64;
    for (int h = 0; h < 2; h++) {
      if (32 * h >= R) break;
      for (int l0 = 0; l0 < 8; l0++) {
        uint32_t ms4 = 0, mt4 = 0;
#pragma unroll
        for (int b = 0; b < NPL; b++) {
          const uint32_t ws = h ? sh[b] : sl[b], wt = h ? th[b] : tl[b];
          ms4 |= ((ws >> l0) & 0x01010101u) << b;
          mt4 |= ((wt >> l0) & 0x01010101u) << b;
        }
        float sv[4];
        int64_t pos[4];
        bool ok[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
          const int l = 32 * h + l0 + 8 * k;
          const int tt = l + c;
          ok[k] = t.jok && l < R;
          const uint32_t ai = (uint32_t)al_s[min(l, 63)];
          const uint32_t ms = (ms4 >> (8 * k)) & 0xFFu, mt = (mt4 >> (8 * k)) & 0xFFu;
          sv[k] = ok[k] ? a.table[tab_index((int)ai, t.bl, (int)ms, (int)mt)] : 0.0f;
          pos[k] = (int64_t)tt * R + l;
          if (ok[k] && a.ms_out) {
            const int64_t cell = d.rm_off + (int64_t)(r0 + l) * m + c;
            a.ms_out[cell] = (int32_t)ms;
            a.mt_out[cell] = (int32_t)mt;
          }
        }
#pragma unroll
        for (int k = 0; k < 4; k++)
          if (ok[k]) strip[pos[k]] = sv[k];
      }
    }
  } else {
    for (int l = 0; l < R; l++) {
      const int ai = al_s[l];
      if (t.jok) {
        const int ms = (int)bs_get<NPL>(sl, sh, l), mt = (int)bs_get<NPL>(tl, th, l);
        const float sv = (ai < kTabLen && t.bl < kTabLen)
                             ? a.table[tab_index(ai, t.bl, ms, mt)]
                             : score_direct(a.w0, a.w1, a.w2, a.w3, ms, ai, mt, t.bl);
        a.S[d.s_off + score_pos(r0 + l, c, n, m)] = sv;
        if (a.ms_out) {
          const int64_t cell = d.rm_off + (int64_t)(r0 + l) * m + c;
          a.ms_out[cell] = ms;
          a.mt_out[cell] = mt;
        }
      }
    }
  }
}

__global__ __launch_bounds__(kTileThreads) void sim_tile_kernel(SimArgs a) {
  __shared__ int32_t ukey[kUcap];
  __shared__ uint16_t ulid[kUcap];
  __shared__ __align__(16) uint16_t tdoc[kTdocCap];
  __shared__ uint8_t tsen[kTdocCap];
  __shared__ uint16_t toff[kJcap];
  __shared__ uint16_t toff_o[kJcap + 1];
  __shared__ uint16_t tlen[kJcap];
  __shared__ uint64_t Dw[kTcap + 4];
  __shared__ uint64_t Bw[kTileWaves][kTcap + 4];
  __shared__ int alw[kTileWaves][64];
  __shared__ int sh_scan[kTileWaves];
  __shared__ int sh_j1;

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

  for (int64_t item = blockIdx.x; item < a.n_items; item += gridDim.x) {
    const SimItem it = a.items[item];
    PairDesc d;  // the descriptor fields the item carries
    d.n = it.n, d.m = it.m, d.src_sent0 = it.src_sent0, d.tgt_sent0 = it.tgt_sent0, d.s_off = it.s_off, d.rm_off = it.rm_off;
    const int m = d.m;
    if (m <= 0 || it.i1 <= it.i0) continue;
    const int64_t *toffs = a.tgt_sent_off + d.tgt_sent0;
    const int64_t *soffs = a.src_sent_off + d.src_sent0;

    for (int j0 = 0; j0 < m;) {
      if (tid < 64) chunk_end(toffs, j0, m, a.n_tgt_tok, &sh_j1, nullptr);
      for (int s = tid; s < kUcap; s += kTileThreads) ukey[s] = kEmpty;
      __syncthreads();
      const int j1 = sh_j1;
      const int nj = j1 - j0;
      const int64_t tbase = clamp64(toffs[j0], 0, a.n_tgt_tok);
      const int ntok = (int)clamp64(clamp64(toffs[j1], 0, a.n_tgt_tok) - tbase, 0, kTcap);
      int blen = 0;
      if (tid < nj) {
        const int ostart = (int)clamp64(clamp64(toffs[j0 + tid], 0, a.n_tgt_tok) - tbase, 0, ntok);
        const int oend = (int)clamp64(clamp64(toffs[j0 + tid + 1], 0, a.n_tgt_tok) - tbase, ostart, ntok);
        blen = oend - ostart;
        toff_o[tid] = (uint16_t)ostart;
        tlen[tid] = (uint16_t)blen;
      }
      int npad;
      const int pstart = block_excl_sum<kTileWaves>((blen + 3) & ~3, sh_scan, &npad);
      if (tid < nj) toff[tid] = (uint16_t)pstart;
      if (tid == 0) toff_o[nj] = (uint16_t)ntok;
      for (int q = tid; q < npad; q += kTileThreads) tdoc[q] = 0xFFFF;
      __syncthreads();
      for (int p = tid; p < ntok; p += kTileThreads) {
        int lo = 0, hi = nj - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (toff_o[mid] <= p)
            lo = mid;
          else
            hi = mid - 1;
        }
        const int32_t x = a.tgt_tok[tbase + p];
        const int q = toff[lo] + (p - toff_o[lo]);
        tdoc[q] = x < 0 ? (uint16_t)0xFFFF : (uint16_t)u_insert(ukey, x);
        tsen[q] = (uint8_t)lo;
      }
      __syncthreads();
      constexpr int kSpt = kUcap / kTileThreads;
      int cnt = 0;
#pragma unroll
      for (int k = 0; k < kSpt; k++) cnt += (ukey[tid * kSpt + k] != kEmpty);
      int total;
      int r = block_excl_sum<kTileWaves>(cnt, sh_scan, &total);
#pragma unroll
      for (int k = 0; k < kSpt; k++) {
        const int s = tid * kSpt + k;
        if (ukey[s] != kEmpty) ulid[s] = (uint16_t)(1 + r++);
      }
      const int nlid = total + 1;
      for (int k = tid; k < nlid; k += kTileThreads) Dw[k] = 0;
      __syncthreads();
      for (int q = tid; q < npad; q += kTileThreads) {
        const uint16_t s = tdoc[q];
        const uint16_t id = s == 0xFFFF ? (uint16_t)0 : ulid[s];
        tdoc[q] = id;
        if (id) atomicOr(reinterpret_cast<unsigned long long *>(&Dw[id]), 1ull << tsen[q]);
      }
      __syncthreads();

      for (int r0 = it.i0 + 64 * wv; r0 < it.i1; r0 += 64 * kTileWaves) {  // 64-row groups of the item
        const int R = min(64, it.i1 - r0);
        TileCtx tc;
        tc.ukey = ukey;
        tc.ulid = ulid;
        tc.D = Dw;
        tc.B = Bw[wv];
        tc.jok = lane < nj;
        tc.bl = tc.jok ? tlen[lane] : 0;
        tc.tp = tdoc + (tc.jok ? toff[lane] : 0);
        tc.nj = nj;
        tc.j0 = j0;
        tc.nlid = nlid;
        // counts above 63 need the wide planes (sentences over 63 tokens)
        int al = 0;
        if (lane < R) {
          const int64_t b0 = clamp64(soffs[r0 + lane], 0, a.n_src_tok);
          al = (int)min<int64_t>(clamp64(soffs[r0 + lane + 1], b0, a.n_src_tok) - b0, 0x7fffffff);
        }
        const bool wide = wave_max(max(al, tc.bl)) > 63;
        if (wide)
          tile_work<kWidePlanes>(a, d, soffs, r0, R, tc, lane, alw[wv]);
        else
          tile_work<kFastPlanes>(a, d, soffs, r0, R, tc, lane, alw[wv]);
      }
      __syncthreads();
      j0 = j1;
    }
  }
}

// ------------------------------------------- (a) similarity, kernels 3 and 4
// Bit-sliced tiles worked by four waves together.  A tile is one 64-row
// strip of a pair (rows r0 .. r0 + R - 1) against one chunk of its target
// sentences (at most 64 sentences and TC tokens; kernel 3 takes TC = 1280,
// three workgroups per CU, kernel 4 TC = 2048, two per CU, which fills the
// chunk's 64 lanes with sentences of the scale workload's lengths).  The
// chunk's distinct target ids get dense local ids through an LDS hash, and
//   D[id] = set of the chunk's sentences holding id (bit j: sentence j0 + j);
// the source pass builds
//   B[id] = set of the strip's rows whose translation set X_i holds id.
// Counts are kept in bit-sliced counters (plane p holds bit p of 64 counts):
//   source pass, lane = row i: for every position q, the OR of D over the
//     translations of s_i[q] is the set of sentences j that meet T(s_i[q]);
//     adding it counts m_s(i, .) for the 64 sentences at once;
//   target pass, lane = sentence j: for every position p, B[id(t_j[p])] is the
//     set of rows whose X_i holds t_j[p]; adding it counts m_t(., j) for the
//     64 rows at once.
// Sets are added four at a time with carry-save adders.  The waves split both
// passes by position (wave w takes source positions q = w mod 4 and target
// positions in blocks 4w .. 4w + 3 mod 16); their partial counters are summed
// through LDS, the m_s planes transposed (lane = sentence), and each wave
// scores a quarter of the tile's rows from the score table.  Tiles whose
// sentences exceed 63 tokens (counts need 11 planes) run both passes on one
// wave and score cell by cell.  A workgroup takes a work item (a pair's rows,
// at most four strips) chunk by chunk: the hash and D of a chunk are built
// once and kept while each of the item's strips is counted against it, with
// B and the counter exchange sharing one region that is cleared per strip.
constexpr int kBitsWaves = 4;
constexpr int kBitsThreads = 64 * kBitsWaves;
constexpr int kBitsNarrow = 6;  // planes for counts <= 63
constexpr int kBitsWide = 11;   // planes for counts <= 2047 (sentences of at most 1024 tokens)

// TC buckets of two slots (load <= 1/2); the bucket of an id is the high
// word of its multiplicative hash times TC.
template <int TC>
struct BitsHash {
  static constexpr uint32_t kNB = TC;
  // groups of four source positions per iteration of the source pass (one:
  // with the chunk's hash and D kept over an item's strips, two groups left
  // the larger chunk size short of registers)
  static constexpr int kGroups = 1;
};
template <int TC>
struct BitsLds {
  // the chunk's id hash (TC buckets of two {key, local id} slots) and D (id 0:
  // none, always 0; one spare entry): built once per chunk, read by every
  // strip of the item
  __align__(16) int2 ent[2 * BitsHash<TC>::kNB];
  __align__(16) uint64_t D[TC + 2];
  // region W, per strip: B during the two passes (with one spare entry per
  // lane after the ids, the target of the lanes whose id is not in the
  // chunk), then the waves' partial counters and the summed and transposed
  // ones, then the tile's scores (row r, chunk sentence j at j + 66 r: both
  // the writes by sentence and the reads by anti-diagonal are free of bank
  // conflicts); while a chunk is staged, the sentence of each staged position
  union {
    uint64_t B[TC + 2 + 64];
    uint64_t xch[2 * (kBitsWaves - 1) * kBitsNarrow * 64];
    uint64_t fin[2 * kBitsWide * 64];
    float stage[66 * 64];
    uint8_t tsen[TC + 3 * kJcap];
  } w;
  __align__(16) uint16_t tdoc[TC + 3 * kJcap];  // local ids, each sentence padded to a multiple of 4 (id 0)
  uint16_t toff[kJcap], toff_o[kJcap + 1], tlen[kJcap];
  int ends[kJcap];
  int j1, nlid, npad, bmax;
};

// The chunk's id hash: NB buckets of two {key, local id} slots, read with one
// 16-byte load.  A key goes to the first free slot from its home bucket on
// (slot 0 before slot 1, then the next bucket); an insert that finds a bucket
// full of other keys marks it (kBitsOverflow in slot 1's id word) before
// moving on.  A search therefore ends at the first bucket that holds its key
// or carries no mark, which for most searches is the home bucket.
constexpr int kBitsOverflow = 1 << 30;
constexpr int kBitsIdMask = 0xFFFF;

template <uint32_t NB>
__device__ __forceinline__ uint32_t bits_bucket(int32_t x) { return __umulhi(hash32(x), NB); }

// Insert target id x (>= 0): its slot (2 bucket + 0 or 1), and whether x was new.
template <uint32_t NB>
__device__ __forceinline__ int bits_insert(int2 *ent, int32_t x, bool &fresh) {
  uint32_t b = bits_bucket<NB>(x);
  for (;;) {  // at most TC distinct keys in 2 TC slots
#pragma unroll
    for (int k = 0; k < 2; k++) {
      const int prev = atomicCAS(&ent[2 * b + k].x, kEmpty, x);
      if (prev == kEmpty || prev == x) {
        fresh = prev == kEmpty;
        return (int)(2 * b + k);
      }
    }
    atomicOr(&ent[2 * b + 1].y, kBitsOverflow);  // searches passing this bucket go on
    b = b + 1 == NB ? 0 : b + 1;
  }
}

// Local ids of K target ids at once (0: not an id of the chunk, or x < 0).
// Every home bucket is read before any further one; the searches that go on
// are tracked in one bit mask per lane, and each round issues all of its
// reads before using any.
template <uint32_t NB, int K>
__device__ __forceinline__ void bits_find(const int4 *ent4, const int32_t (&x)[K], int (&lid)[K]) {
  static_assert(K <= 32, "pending searches are one bit each");
  uint32_t b[K];
  int4 e[K];
#pragma unroll
  for (int k = 0; k < K; k++) {
    b[k] = bits_bucket<NB>(x[k]);
    e[k] = ent4[b[k]];
  }
  // Branch-free on the first round: a key sits in at most one slot, and a
  // search for x < 0 gets 0 (an empty slot's id word is 0, and only a full
  // bucket carries the mark).
  uint32_t pend = 0;
#pragma unroll
  for (int k = 0; k < K; k++) {
    const uint32_t v = (e[k].x == x[k] ? (uint32_t)e[k].y : 0u) | (e[k].z == x[k] ? (uint32_t)e[k].w : 0u);
    lid[k] = (int)(v & kBitsIdMask);
    pend |= (uint32_t)((x[k] >= 0) & (lid[k] == 0) & ((e[k].w & kBitsOverflow) != 0)) << k;
  }
  while (pend) {
#pragma unroll
    for (int k = 0; k < K; k++) b[k] = ((pend >> k) & 1u) ? (b[k] + 1 == NB ? 0 : b[k] + 1) : b[k];
#pragma unroll
    for (int k = 0; k < K; k++)
      if ((pend >> k) & 1u) e[k] = ent4[b[k]];
#pragma unroll
    for (int k = 0; k < K; k++) {
      if ((pend >> k) & 1u) {
        lid[k] = e[k].x == x[k] ? (e[k].y & kBitsIdMask) : e[k].z == x[k] ? (e[k].w & kBitsIdMask) : 0;
        if (lid[k] != 0 || (e[k].w & kBitsOverflow) == 0) pend &= ~(1u << k);
      }
    }
  }
}

// Carry-save adder: a + b + c = s + 2 carry, bit by bit.
__device__ __forceinline__ void bits_csa(uint32_t &s, uint32_t &carry, uint32_t a, uint32_t b, uint32_t c) {
  const uint32_t t = a ^ b;
  s = t ^ c;
  carry = (t & c) | (~t & a);
}

// Add four sets (one bit per counter) into NPL bit-sliced planes.  The caller
// guarantees that no count exceeds 2^NPL - 1.
template <int NPL>
__device__ __forceinline__ void bits_add4(uint32_t (&P)[NPL], uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3) {
  uint32_t s, ca, cb, c4;
  bits_csa(s, ca, P[0], x0, x1);     // P0 + x0 + x1 = s + 2 ca
  bits_csa(P[0], cb, s, x2, x3);     // s + x2 + x3 = P0' + 2 cb
  bits_csa(P[1], c4, P[1], ca, cb);  // P1 + ca + cb = P1' + 2 c4
#pragma unroll
  for (int k = 2; k < NPL; k++) {
    const uint32_t t = P[k] & c4;
    P[k] ^= c4;
    c4 = t;
  }
}

// P += Q, counter by counter (ripple carry over the planes).
template <int NPL>
__device__ __forceinline__ void bits_add_counters(uint32_t (&P)[NPL], const uint32_t (&Q)[NPL]) {
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < NPL; k++) {
    uint32_t s, cn;
    bits_csa(s, cn, P[k], Q[k], c);
    P[k] = s;
    c = cn;
  }
}

// End of the target chunk starting at sentence j0: the largest j1 <= j0 + 64
// whose sentences [j0, j1) hold at most TC tokens (at least one sentence);
// lane L of the calling wave also keeps the end of the chunk's sentence L
// relative to the chunk's first token (clamped to [0, 2^30]).
template <int TC>
__device__ __forceinline__ void bits_chunk_end(const int64_t *toffs, int j0, int m, int64_t n_tok, int *out, int *ends) {
  const int lane = threadIdx.x & 63;
  const int64_t base = clamp64(toffs[j0], 0, n_tok);
  const int jj = j0 + 1 + lane;
  const bool ok = jj <= min(m, j0 + kJcap);
  const int64_t e = ok ? clamp64(toffs[jj], 0, n_tok) - base : 0;
  const uint64_t bal = __ballot(ok && e <= TC);
  const int lead = ~bal == 0 ? 64 : __builtin_ctzll(~bal);
  if (lane == 0) *out = j0 + max(1, lead);
  ends[lane] = (int)clamp64(e, 0, 1 << 30);
}

// Translation records of iteration u of the source pass (below): positions
// q = q0 + qs (NR u + k) of this lane's row, {-1, -1, -1, -1} past its end.
template <int NR>
__device__ __forceinline__ void bits_s_fetch(const SimArgs &a, int64_t sb, int al, int q0, int qs, int u,
                                             int4 (&r)[NR]) {
#pragma unroll
  for (int k = 0; k < NR; k++) {
    const int q = q0 + qs * (NR * u + k);
    r[k] = q < al ? a.trans[sb + q] : make_int4(-1, -1, -1, -1);
  }
}

// Source pass over the positions q = q0 + qs (4 G u + k) of this lane's row
// (record base sb, length al; amax: the longest row of the strip): marks B and
// adds, per position, the set of the chunk's sentences meeting its
// translations into the planes (lo: sentences 0-31, hi: 32-63).  G groups of
// four positions per iteration (their lookups overlap); ra holds the first
// iteration's records (fetched by the caller), and the next iteration's are
// fetched while one is worked on.
template <int NPL, int TC, int G>
__device__ __forceinline__ void bits_s_pass(const SimArgs &a, BitsLds<TC> &L, int64_t sb, int al, int amax, int q0,
                                            int qs, int4 (&ra)[4 * G], uint32_t (&lo)[NPL], uint32_t (&hi)[NPL]) {
  constexpr uint32_t HB = BitsHash<TC>::kNB;  // buckets of two slots
  constexpr int NR = 4 * G;                   // records per iteration
  const int4 *ent4 = reinterpret_cast<const int4 *>(L.ent);
  const int lane = threadIdx.x & 63;
  const unsigned long long rowbit = 1ull << lane;
  unsigned long long *B = reinterpret_cast<unsigned long long *>(L.w.B);
  const uint64_t *D = L.D;
  for (int u = 0; q0 + qs * NR * u < amax; u++) {
    int4 rb[NR];
    bits_s_fetch<NR>(a, sb, al, q0, qs, u + 1, rb);
    bool far = false;
    uint64_t c[NR];
#pragma unroll
    for (int hf = 0; hf < NR / 2; hf++) {  // two records at a time (register pressure)
      int32_t x[8];
#pragma unroll
      for (int k = 0; k < 2; k++) {
        const int4 rr = ra[2 * hf + k];
        const bool f = rr.x == -2;  // more than four translations: looked up below
        far |= f;
        x[4 * k] = f ? -1 : rr.x;
        x[4 * k + 1] = f ? -1 : rr.y;
        x[4 * k + 2] = f ? -1 : rr.z;
        x[4 * k + 3] = f ? -1 : rr.w;
      }
      int lid[8];
      bits_find<HB>(ent4, x, lid);
      // ids not in the chunk are marked in the lane's own spare entry (one
      // shared slot would serialise the atomics), so no lane branches
#pragma unroll
      for (int k = 0; k < 8; k++) atomicOr(&B[lid[k] ? lid[k] : TC + 2 + lane], rowbit);
#pragma unroll
      for (int k = 0; k < 2; k++)
        c[2 * hf + k] = (D[lid[4 * k]] | D[lid[4 * k + 1]]) | (D[lid[4 * k + 2]] | D[lid[4 * k + 3]]);
    }
    if (far) {
#pragma unroll
      for (int k = 0; k < NR; k++) {
        if (ra[k].x == -2) {
          for (int e = 0; e < ra[k].z; e++) {
            const int32_t y[1] = {a.lex.vals[ra[k].y + e]};
            int l[1];
            bits_find<HB>(ent4, y, l);
            if (l[0]) atomicOr(&B[l[0]], rowbit);
            c[k] |= D[l[0]];
          }
        }
      }
    }
#pragma unroll
    for (int g = 0; g < G; g++) {
      bits_add4<NPL>(lo, (uint32_t)c[4 * g], (uint32_t)c[4 * g + 1], (uint32_t)c[4 * g + 2], (uint32_t)c[4 * g + 3]);
      bits_add4<NPL>(hi, (uint32_t)(c[4 * g] >> 32), (uint32_t)(c[4 * g + 1] >> 32), (uint32_t)(c[4 * g + 2] >> 32),
                     (uint32_t)(c[4 * g + 3] >> 32));
    }
#pragma unroll
    for (int k = 0; k < NR; k++) ra[k] = rb[k];
  }
}

template <int NPL, int TC>
__device__ __forceinline__ void bits_t_pass(const BitsLds<TC> &L, int nj, int k0, int ks, uint32_t (&lo)[NPL],
                                            uint32_t (&hi)[NPL]) {
  const int j = threadIdx.x & 63;
  const bool jok = j < nj;
  const int bl = jok ? L.tlen[j] : 0;
  const uint16_t *tp = L.tdoc + (jok ? L.toff[j] : 0);
  const uint64_t *B = L.w.B;
  const int bmax = L.bmax;
  for (int k = k0; k < bmax; k += 2 * ks) {
    uint64_t x[8];
#pragma unroll
    for (int g = 0; g < 2; g++) {
      const int kk = k + g * ks;
      uint2 ids = make_uint2(0u, 0u);  // id 0: B[0] = 0
      if (kk < bl) ids = *reinterpret_cast<const uint2 *>(tp + kk);
      x[4 * g] = B[ids.x & 0xFFFFu];
      x[4 * g + 1] = B[ids.x >> 16];
      x[4 * g + 2] = B[ids.y & 0xFFFFu];
      x[4 * g + 3] = B[ids.y >> 16];
    }
#pragma unroll
    for (int g = 0; g < 2; g++) {
      bits_add4<NPL>(lo, (uint32_t)x[4 * g], (uint32_t)x[4 * g + 1], (uint32_t)x[4 * g + 2], (uint32_t)x[4 * g + 3]);
      bits_add4<NPL>(hi, (uint32_t)(x[4 * g] >> 32), (uint32_t)(x[4 * g + 1] >> 32), (uint32_t)(x[4 * g + 2] >> 32),
                     (uint32_t)(x[4 * g + 3] >> 32));
    }
  }
}

// Transpose a 64 x 64 bit matrix held one row per lane (lo: columns 0-31,
// hi: 32-63); afterwards lane c holds column c.  The six exchange stages use
// lane moves that stay in the VALU: the lane-half swap for distance 32, the
// row-pair swap for 16, and DPP mirrors and quad permutes for 8, 4, 2, 1.
__device__ __forceinline__ uint32_t bits_xor_lane(uint32_t v, int d) {
  switch (d) {
    case 1: return dpp_mov<0xB1>(v);                  // quad_perm [1, 0, 3, 2]
    case 2: return dpp_mov<0x4E>(v);                  // quad_perm [2, 3, 0, 1]
    case 4: return dpp_mov<0x1B>(dpp_mov<0x141>(v));  // half-row mirror, then quad_perm [3, 2, 1, 0]
    default: return dpp_mov<0x141>(dpp_mov<0x140>(v));  // row mirror, then half-row mirror (distance 8)
  }
}

__device__ __forceinline__ void bits_transpose64(uint32_t &lo, uint32_t &hi, int lane) {
  {  // distance 32: lanes 0-31 take the low words of lanes 32-63 as their high words and vice versa
    const auto r = __builtin_amdgcn_permlane32_swap(lo, hi, false, false);
    lo = r[0];
    hi = r[1];
  }
  {  // distance 16 (inside each 32-lane half): the lower lane of a pair swaps its high 16 bits with
     // the upper lane's low 16 bits
    const bool up = (lane & 16) != 0;
    const uint32_t xl = up ? (lo & 0xFFFFu) : (lo >> 16), xh = up ? (hi & 0xFFFFu) : (hi >> 16);
    const auto rl = __builtin_amdgcn_permlane16_swap(xl, xl, false, false);
    const auto rh = __builtin_amdgcn_permlane16_swap(xh, xh, false, false);
    const uint32_t yl = up ? rl[0] : rl[1], yh = up ? rh[0] : rh[1];
    lo = up ? ((lo & 0xFFFF0000u) | yl) : ((lo & 0xFFFFu) | (yl << 16));
    hi = up ? ((hi & 0xFFFF0000u) | yh) : ((hi & 0xFFFFu) | (yh << 16));
  }
#pragma unroll
  for (int s = 8; s >= 1; s >>= 1) {
    const uint32_t m = s == 8 ? 0x00FF00FFu : s == 4 ? 0x0F0F0F0Fu : s == 2 ? 0x33333333u : 0x55555555u;
    const uint32_t ylo = bits_xor_lane(lo, s), yhi = bits_xor_lane(hi, s);
    const bool up = (lane & s) != 0;
    const uint32_t alo = (lo & m) | ((ylo & m) << s), ahi = (hi & m) | ((yhi & m) << s);
    const uint32_t blo = (lo & ~m) | ((ylo & ~m) >> s), bhi = (hi & ~m) | ((yhi & ~m) >> s);
    lo = up ? blo : alo;
    hi = up ? bhi : ahi;
  }
}

template <int NPL>
__device__ __forceinline__ void bits_store(uint64_t *dst, const uint32_t (&lo)[NPL], const uint32_t (&hi)[NPL]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int p = 0; p < NPL; p++) dst[p * 64 + lane] = ((uint64_t)hi[p] << 32) | lo[p];
}

template <int NPL>
__device__ __forceinline__ void bits_load(const uint64_t *src, uint32_t (&lo)[NPL], uint32_t (&hi)[NPL]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int p = 0; p < NPL; p++) {
    const uint64_t v = src[p * 64 + lane];
    lo[p] = (uint32_t)v;
    hi[p] = (uint32_t)(v >> 32);
  }
}

template <int TC>
__global__ __launch_bounds__(kBitsThreads, TC <= 1280 ? 3 : 2) void sim_bits_kernel(SimArgs a) {
  static_assert(kMaxItemRows <= 4 * 64, "an item's rows are kept for at most four strips");
  __shared__ BitsLds<TC> L;
  constexpr uint32_t NS = 2 * BitsHash<TC>::kNB;  // hash slots
  constexpr int kTpt = (TC + kBitsThreads - 1) / kBitsThreads;  // staged tokens per thread
  constexpr int NR = 4 * BitsHash<TC>::kGroups;                 // source records per pass iteration
  constexpr int kPl = kBitsNarrow * 64;                         // one set of narrow planes in W
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);

  for (int64_t item = blockIdx.x; item < a.n_items; item += gridDim.x) {
    const SimItem it = a.items[item];
    const int n = it.n, m = it.m;
    if (m <= 0 || it.i1 <= it.i0) continue;
    const int64_t *toffs = a.tgt_sent_off + it.tgt_sent0;
    const int64_t *soffs = a.src_sent_off + it.src_sent0;
    // this lane's row of each of the item's strips (every wave holds a strip's
    // rows in the same lanes); items start on a strip and span at most four
    int64_t sbv[4];
    int alv[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int r = it.i0 + 64 * k + lane;
      sbv[k] = 0;
      alv[k] = 0;
      if (r < it.i1) {
        sbv[k] = clamp64(soffs[r], 0, a.n_src_tok);
        alv[k] = (int)min(clamp64(soffs[r + 1], sbv[k], a.n_src_tok) - sbv[k], (int64_t)0x7fffffff);
      }
    }

    for (int j0 = 0; j0 < m;) {
      // ---- stage the chunk once for all of the item's strips: ids -> local ids, sentences, D ----
      if (tid < 64) bits_chunk_end<TC>(toffs, j0, m, a.n_tgt_tok, &L.j1, L.ends);
      if (tid == 0) L.nlid = 0;
      {  // 16-byte stores: the hash to {empty, 0}, D to 0
        int4 *e4 = reinterpret_cast<int4 *>(L.ent);
        for (int s = tid; s < (int)NS / 2; s += kBitsThreads) e4[s] = make_int4(kEmpty, 0, kEmpty, 0);
        uint4 *d4 = reinterpret_cast<uint4 *>(L.D);
        for (int s = tid; s < (TC + 2) / 2; s += kBitsThreads) d4[s] = make_uint4(0u, 0u, 0u, 0u);
      }
      __syncthreads();
      const int j1 = L.j1, nj = j1 - j0;
      const int64_t tbase = clamp64(toffs[j0], 0, a.n_tgt_tok);
      const int ntok = min(L.ends[nj - 1], TC);
      int32_t xs[kTpt];
#pragma unroll
      for (int u = 0; u < kTpt; u++) {
        const int p = tid + kBitsThreads * u;
        xs[u] = p < ntok ? a.tgt_tok[tbase + p] : -1;
      }
      if (tid < 64) {  // sentence layout by one wave-wide scan
        int ostart = 0, blen = 0;
        if (lane < nj) {
          ostart = lane == 0 ? 0 : min(L.ends[lane - 1], ntok);
          blen = min(max(L.ends[lane], ostart), ntok) - ostart;
        }
        const int plen = (blen + 3) & ~3;
        int x = plen;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int y = __shfl_up(x, o);
          if (lane >= o) x += y;
        }
        const int pstart = x - plen;
        if (lane < nj) {
          L.toff_o[lane] = (uint16_t)ostart;
          L.tlen[lane] = (uint16_t)blen;
          L.toff[lane] = (uint16_t)pstart;
          for (int q = blen; q < plen; q++) L.tdoc[pstart + q] = 0xFFFF;
        }
        if (lane == 0) L.toff_o[nj] = (uint16_t)ntok;
        if (lane == 63) L.npad = x;
        const int bm = wave_max(blen);
        if (lane == 0) L.bmax = bm;
      }
      __syncthreads();
      // every token into the hash; a key new to the chunk takes the next local id
#pragma unroll
      for (int u = 0; u < kTpt; u++) {
        const int p = tid + kBitsThreads * u;
        bool fresh = false;
        int h = 0xFFFF;
        if (p < ntok) {
          int lo = 0;  // sentence holding token p: the last start <= p
#pragma unroll
          for (int step = kJcap / 2; step >= 1; step >>= 1)
            if (lo + step < nj && L.toff_o[lo + step] <= p) lo += step;
          const int dst = L.toff[lo] + (p - L.toff_o[lo]);
          if (xs[u] >= 0) h = bits_insert<BitsHash<TC>::kNB>(L.ent, xs[u], fresh);
          L.tdoc[dst] = (uint16_t)h;
          L.w.tsen[dst] = (uint8_t)lo;
        }
        const uint64_t nb = __ballot(fresh);
        if (nb) {
          const int lead = __builtin_ctzll(nb);
          int base = 0;
          if (lane == lead) base = atomicAdd(&L.nlid, __popcll(nb));
          base = __builtin_amdgcn_readlane(base, lead);
          if (fresh) atomicOr(&L.ent[h].y, 1 + base + __popcll(nb & ((1ull << lane) - 1)));  // keeps a mark
        }
      }
      __syncthreads();
      const int npad = L.npad;
      for (int q = tid; q < npad; q += kBitsThreads) {
        const uint16_t s = L.tdoc[q];
        const int id = s == 0xFFFF ? 0 : (L.ent[s].y & kBitsIdMask);
        L.tdoc[q] = (uint16_t)id;
        if (id) atomicOr(reinterpret_cast<unsigned long long *>(&L.D[id]), 1ull << L.w.tsen[q]);
      }
      __syncthreads();  // the hash, D and the staged ids are complete; W is free
      const int bmax = L.bmax;

      const int jj = lane;  // this lane's sentence in the scoring stage
      const bool jok = jj < nj;
      const int bj = jok ? L.tlen[jj] : 0;
      const int c = j0 + jj;
      for (int sx = 0, r0 = it.i0; r0 < it.i1; sx++, r0 += 64) {
        const int R = min(64, n - r0);
        float *const strip = a.S + it.s_off + (int64_t)(r0 >> 6) * (m + 63) * 64;
        int64_t sb = sbv[0];
        int al = alv[0];
#pragma unroll
        for (int k = 1; k < 4; k++)
          if (sx == k) {
            sb = sbv[k];
            al = alv[k];
          }
        const int amax = __builtin_amdgcn_readfirstlane(wave_max(al));
        const bool narrow = amax < 64 && bmax < 64;
        // the source pass's first records travel while B is cleared
        int4 ra[NR];
        bits_s_fetch<NR>(a, sb, al, narrow ? wv : 0, narrow ? kBitsWaves : 1, 0, ra);
        {
          uint4 *b4 = reinterpret_cast<uint4 *>(L.w.B);
          for (int s = tid; s < (TC + 2) / 2; s += kBitsThreads) b4[s] = make_uint4(0u, 0u, 0u, 0u);
        }
        __syncthreads();
        if (narrow) {
          uint32_t slo[kBitsNarrow] = {}, shi[kBitsNarrow] = {}, tlo[kBitsNarrow] = {}, thi[kBitsNarrow] = {};
          bits_s_pass<kBitsNarrow, TC, BitsHash<TC>::kGroups>(a, L, sb, al, amax, wv, kBitsWaves, ra, slo, shi);
          __syncthreads();  // B complete
          bits_t_pass<kBitsNarrow>(L, nj, 4 * wv, 4 * kBitsWaves, tlo, thi);
          __syncthreads();  // B no longer read: W takes the partial counters
          // W: source partials of waves 1-3 at 0, 1, 2 kPl; target partials of waves 0, 2, 3 at 3, 4, 5 kPl
          uint64_t *const xs_s = L.w.xch, *const xs_t = L.w.xch + (kBitsWaves - 1) * kPl;
          if (wv > 0) bits_store<kBitsNarrow>(xs_s + (wv - 1) * kPl, slo, shi);
          if (wv != 1) bits_store<kBitsNarrow>(xs_t + (wv == 0 ? 0 : wv - 1) * kPl, tlo, thi);
          __syncthreads();
          // each sum goes where its wave read its own first partial set: summed m_s
          // (lane = row) at 0, m_t (lane = sentence) at 3 kPl
          uint64_t *const comb_s = L.w.xch, *const fin_t = xs_t, *const fin_s = L.w.xch + kPl;
          if (wv == 0) {
            for (int w = 0; w < kBitsWaves - 1; w++) {
              uint32_t ql[kBitsNarrow], qh[kBitsNarrow];
              bits_load<kBitsNarrow>(xs_s + w * kPl, ql, qh);
              bits_add_counters<kBitsNarrow>(slo, ql);
              bits_add_counters<kBitsNarrow>(shi, qh);
            }
            bits_store<kBitsNarrow>(comb_s, slo, shi);
          } else if (wv == 1) {
            for (int w = 0; w < kBitsWaves - 1; w++) {
              uint32_t ql[kBitsNarrow], qh[kBitsNarrow];
              bits_load<kBitsNarrow>(xs_t + w * kPl, ql, qh);
              bits_add_counters<kBitsNarrow>(tlo, ql);
              bits_add_counters<kBitsNarrow>(thi, qh);
            }
            bits_store<kBitsNarrow>(fin_t, tlo, thi);
          }
          __syncthreads();
          // transpose m_s (lane = sentence) into the consumed partials of wave 2:
          // wave w takes planes w and w + 4
          for (int p = wv; p < kBitsNarrow; p += kBitsWaves) {
            const uint64_t v = comb_s[p * 64 + lane];
            uint32_t vl = (uint32_t)v, vh = (uint32_t)(v >> 32);
            bits_transpose64(vl, vh, lane);
            fin_s[p * 64 + lane] = ((uint64_t)vh << 32) | vl;
          }
          __syncthreads();
          // score: wave w takes rows 32 h + l0 + 8 k with l0 = 2 w, 2 w + 1;
          // all sixteen table reads are issued before the first store
          uint32_t sl[kBitsNarrow], sh[kBitsNarrow], tl[kBitsNarrow], th[kBitsNarrow];
          bits_load<kBitsNarrow>(fin_s, sl, sh);
          bits_load<kBitsNarrow>(fin_t, tl, th);
          __syncthreads();  // the counters are in registers: W takes the scores
          float sv[16];
#pragma unroll
          for (int g = 0; g < 4; g++) {
            const int h = g >> 1, l0 = 2 * wv + (g & 1);
            uint32_t ms4 = 0, mt4 = 0;
#pragma unroll
            for (int p = 0; p < kBitsNarrow; p++) {
              ms4 |= (((h ? sh[p] : sl[p]) >> l0) & 0x01010101u) << p;
              mt4 |= (((h ? th[p] : tl[p]) >> l0) & 0x01010101u) << p;
            }
#pragma unroll
            for (int k = 0; k < 4; k++) {
              const int r = 32 * h + l0 + 8 * k;
              const bool ok = jok && r < R;
              const int ar = __builtin_amdgcn_readlane(al, r);  // wave-uniform row
              const uint32_t ms = (ms4 >> (8 * k)) & 0xFFu, mt = (mt4 >> (8 * k)) & 0xFFu;
              sv[4 * g + k] = ok ? a.table[tab_index(ar, bj, (int)ms, (int)mt)] : 0.0f;
              if (ok && a.ms_out) {
                const int64_t cell = it.rm_off + (int64_t)(r0 + r) * m + c;
                a.ms_out[cell] = (int32_t)ms;
                a.mt_out[cell] = (int32_t)mt;
              }
            }
          }
          // the scores go out by anti-diagonal through W (lane = row), so each
          // store writes consecutive slots of the strip
          float *const stage = L.w.stage;
#pragma unroll
          for (int g = 0; g < 4; g++) {
#pragma unroll
            for (int k = 0; k < 4; k++) stage[jj + 66 * (32 * (g >> 1) + 2 * wv + (g & 1) + 8 * k)] = sv[4 * g + k];
          }
          __syncthreads();
          for (int d = wv; d < nj + R - 1; d += kBitsWaves) {
            const int jl = d - lane;  // this lane's sentence on the diagonal
            if (lane < R && jl >= 0 && jl < nj) strip[(int64_t)(j0 + d) * R + lane] = stage[jl + 66 * lane];
          }
        } else {
          // sentences of more than 63 tokens: one wave counts, in 11 planes
          uint64_t *const fin_s = L.w.fin, *const fin_t = L.w.fin + kBitsWide * 64;
          if (wv == 0) {
            uint32_t slo[kBitsWide] = {}, shi[kBitsWide] = {}, tlo[kBitsWide] = {}, thi[kBitsWide] = {};
            int4 r4[4];
#pragma unroll
            for (int k = 0; k < 4; k++) r4[k] = ra[k];
            bits_s_pass<kBitsWide, TC, 1>(a, L, sb, al, amax, 0, 1, r4, slo, shi);
            wave_sync();
            bits_t_pass<kBitsWide>(L, nj, 0, 4, tlo, thi);
#pragma unroll
            for (int p = 0; p < kBitsWide; p++) bits_transpose64(slo[p], shi[p], lane);
            wave_sync();  // B reads done before W is overwritten
            bits_store<kBitsWide>(fin_s, slo, shi);
            bits_store<kBitsWide>(fin_t, tlo, thi);
          }
          __syncthreads();
          uint32_t sl[kBitsWide], sh[kBitsWide], tl[kBitsWide], th[kBitsWide];
          bits_load<kBitsWide>(fin_s, sl, sh);
          bits_load<kBitsWide>(fin_t, tl, th);
          for (int r = wv; r < R; r += kBitsWaves) {
            uint32_t ms = 0, mt = 0;
#pragma unroll
            for (int p = 0; p < kBitsWide; p++) {
              ms |= (((r < 32 ? sl[p] >> r : sh[p] >> (r - 32))) & 1u) << p;
              mt |= (((r < 32 ? tl[p] >> r : th[p] >> (r - 32))) & 1u) << p;
            }
            const int ar = __builtin_amdgcn_readlane(al, r);
            if (jok) {
              const float sv = (ar < kTabLen && bj < kTabLen)
                                   ? a.table[tab_index(ar, bj, (int)ms, (int)mt)]
                                   : score_direct(a.w0, a.w1, a.w2, a.w3, (int)ms, ar, (int)mt, bj);
              strip[(r + c) * R + r] = sv;
              if (a.ms_out) {
                const int64_t cell = it.rm_off + (int64_t)(r0 + r) * m + c;
                a.ms_out[cell] = (int32_t)ms;
                a.mt_out[cell] = (int32_t)mt;
              }
            }
          }
        }
        __syncthreads();  // W is cleared for the next strip; the hash and D for the next chunk
      }
      j0 = j1;
    }
  }
}

// Row-major <-> strip-diagonal copies of whole score blocks (parity entries).
__global__ __launch_bounds__(256) void relayout_kernel(const PairDesc *descs, int64_t n_pairs, const float *src,
                                                       float *dst, int to_diag) {
  const int64_t p = blockIdx.y;
  if (p >= n_pairs) return;
  const PairDesc d = descs[p];
  const int64_t cells = (int64_t)d.n * d.m;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < cells; k += (int64_t)gridDim.x * 256) {
    const int i = (int)(k / d.m), c = (int)(k % d.m);
    const int64_t q = score_pos(i, c, d.n, d.m);
    if (to_diag)
      dst[d.s_off + q] = src[d.rm_off + k];
    else
      dst[d.rm_off + k] = src[d.s_off + q];
  }
}

// One wave per document pair.  Rows are taken in strips of 64 (lane l owns
// DP row 64*s + l + 1); the strip sweeps the columns along anti-diagonals:
// at step t lane l computes column j = t - l.  The value from the row above
// arrives from lane l-1 through a one-lane DPP shift; lane 0 reads it from the
// previous strip's bottom row (or the top boundary, built by repeated
// addition).  Scores are prefetched 16 steps ahead into registers.
// Direction codes (D=0, U=1, L=2) are packed 16 per word, row-major, in LDS
// when the pair fits, else in global scratch.  Lane 0 then walks the path
// back from (n, m), writing the D cells backwards into the pair's output
// slots; the wave reads their scores, keeps those >= tau and compacts them in
// path order to the front of the slots.

constexpr int kNwUnroll = 16;
// Word 3 of a raw buffer resource on gfx9-family GPUs (32-bit data format).
constexpr int kBufferFlags = 0x00020000;

struct NwLane {
  float h, upv, topv;
  uint32_t dw;
};

// Hand-off of strip bottom rows between the waves of one workgroup that
// sweeps a large pair with several waves (strip s on wave s mod W): the slot
// of wave w holds (strip << 32) | (columns of that strip's bottom row
// published so far).  A default-constructed pipe (no slots) is the one-wave
// sweep, where strips run in order and nothing is waited for.
struct NwPipe {
  int64_t *prog = nullptr;  // LDS slots, one per wave
  int W = 1;
  int *abort = nullptr;  // LDS flag: a wait ran past its time limit
  uint64_t limit = kNwWaitTicks;  // ticks of the 100 MHz constant counter; 0: give up at once
  // persistent-grid sweep (tagged boundary rows): this launch's tag and the
  // pair's give-up flag in global memory
  uint32_t tag = 0;
  int32_t *gabort = nullptr;
};

// Wait until strip `strip` has published at least `cols` columns (or has been
// finished and its wave moved on).  Wave-uniform; false if the limit was hit.
// After a give-up every later wait of the workgroup returns false at once, so
// the waves finish their sweeps (on stale boundary values, every access still
// inside its arrays) and the pair is reported as failed.
__device__ __forceinline__ bool nw_wait(const NwPipe &pp, int strip, int cols) {
  int64_t *slot = pp.prog + (strip % pp.W);
  if (pp.limit == 0) {  // failure injection: every wait gives up
    __hip_atomic_store(pp.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    return false;
  }
  const uint64_t t0 = wall_clock64();
  for (;;) {
    const int64_t v = __hip_atomic_load(slot, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
    const int vs = (int)(v >> 32), vc = (int)(uint32_t)v;
    if (vs > strip || (vs == strip && vc >= cols)) return true;
    if (__hip_atomic_load(pp.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) return false;
    if (wall_clock64() - t0 > pp.limit) {
      __hip_atomic_store(pp.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// Entry t of the previous strip's bottom row in the persistent-grid sweep,
// for the lanes with `need`, given v, that entry as loaded one block earlier.
// Entries are 8 bytes, {H, tag}, stored with one atomic store by the wave of
// that strip (possibly on another CU or XCD): an entry carrying this launch's
// tag holds this launch's value, so no flag or fence is needed.  The wave
// reads the entries again until every needed one has the tag, for at most the
// time limit; a give-up (or an earlier one for the same pair) sets the pair's
// flag, and the sweep goes on with whatever the entries hold.
__device__ __forceinline__ float nw_row_take(const NwPipe &pp, const uint64_t *row, int t, bool need, uint64_t v) {
  if (pp.limit == 0) {  // failure injection: every wait gives up
    if ((threadIdx.x & 63) == 0) __hip_atomic_store(pp.gabort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return 0.0f;
  }
  bool ok = !need || (uint32_t)(v >> 32) == pp.tag;
  if (__builtin_expect(__ballot(!ok) != 0ull, 0)) {
    const uint64_t t0 = wall_clock64();
    for (;;) {
      const int given_up =
          __builtin_amdgcn_readfirstlane(__hip_atomic_load(pp.gabort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      if (given_up) break;
      if (wall_clock64() - t0 > pp.limit) {
        if ((threadIdx.x & 63) == 0) __hip_atomic_store(pp.gabort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
      if (!ok) {
        v = __hip_atomic_load(row + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = (uint32_t)(v >> 32) == pp.tag;
      }
      if (__ballot(!ok) == 0ull) break;
    }
  }
  return __uint_as_float((uint32_t)v);
}

// Publish `cols` columns of strip `strip`'s bottom row (after this wave's row stores).
__device__ __forceinline__ void nw_publish(const NwPipe &pp, int strip, int cols) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  if ((threadIdx.x & 63) == 0)
    __hip_atomic_store(pp.prog + (strip % pp.W), ((int64_t)strip << 32) | (uint32_t)cols, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Scores of the next 16 steps for this lane: step t reads slot
// (t - 1) * R + lane of the strip (anti-diagonal t - 1).  The strip is read
// through a buffer resource whose range is the strip, so reads before its
// first or after its last slot return 0 without touching memory; the values
// of lanes outside a diagonal are never used.  For strips after the first,
// lane k also fetches the previous strip's bottom-row value H[64s][t] of the
// block's step k (handed to lane 0 by readlane).  In the persistent-grid
// sweep those entries were loaded one block earlier (pend) and are checked
// here, and the next block's are loaded, so a round trip to another CU's
// writes overlaps a block of steps.
template <bool kTagged>
__device__ __forceinline__ void nw_prefetch(float (&buf)[kNwUnroll], float &rbv, __amdgpu_buffer_rsrc_t rs,
                                            const float *rowbuf, bool use_row, int &d, int lane, int R, int m,
                                            const NwPipe &pp, int s, uint64_t &pend) {
  const int t = d + 1 + lane;
  if (kTagged) {
    rbv = 0.0f;
    if (use_row) {
      const uint64_t *row = (const uint64_t *)rowbuf;
      rbv = nw_row_take(pp, row, t, lane < kNwUnroll && t <= m, pend);
      const int tn = t + kNwUnroll;
      pend = (lane < kNwUnroll && tn <= m) ? __hip_atomic_load(row + tn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                            : 0ull;
    }
  } else {
    if (pp.prog && use_row) nw_wait(pp, s - 1, min(m, d + kNwUnroll) + 1);
    rbv = (use_row && lane < kNwUnroll && t <= m) ? rowbuf[t] : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < kNwUnroll; k++) {
    buf[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (d * R + lane) * 4, 0, 0));
    d++;
  }
}

// 16 steps of the strip sweep (t0 a multiple of 16).  Lane l holds DP row
// i = 64s + l + 1 and computes column j = t - l at step t.  Steps with j < 0
// or j > m (and rows past n) compute values that are never read: column 0
// (j = 0) depends only on the lane above, and a lane only ever reads the lane
// above at the column it is itself computing.  Direction codes are packed by
// step: bits 2k..2k+1 of a lane's word hold the code of its cell at step
// t0 + k, and every lane stores its word once per block.  The last row's H
// values are kept in registers and handed to the next strip at the block end.
template <bool kTail, bool kTop, bool kTagged>
__device__ __forceinline__ void nw_steps(const float (&buf)[kNwUnroll], float rbv, int t0, int tend, NwLane &L,
                                         int lane, int i, bool rowok, int lastlane, bool keep_row, int m, int Wr,
                                         float g, uint32_t *dirs, float *rowbuf, const NwPipe &pp, int s) {
  float hb[kNwUnroll];
  if (kTail) {
#pragma unroll
    for (int k = 0; k < kNwUnroll; k++) hb[k] = 0.0f;
  }
  uint32_t dw = 0;
#pragma unroll
  for (int k = 0; k < kNwUnroll; k++) {
    const int t = t0 + k;
    if (kTail && t > tend) break;
    float up0;
    if (kTop) {
      L.topv = __fadd_rn(L.topv, g);  // H[0][t] (starts at -g: -g + g = +0 at t = 0)
      up0 = L.topv;
    } else {
      up0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rbv), k));
    }
    // lane l takes lane l - 1's H (wave_shr:1); lane 0, with no lane below
    // it, keeps the DPP's old value, the row above the strip
    const float up =
        __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(up0), __float_as_int(L.h), 0x138, 0xF, 0xF, false));
    const float dd = __fadd_rn(L.upv, buf[k]);
    const float uu = __fadd_rn(up, g);
    const float ll = __fadd_rn(L.h, g);
    const bool u_wins = uu > dd;
    float best = u_wins ? uu : dd;
    uint32_t code = u_wins ? 1u : 0u;
    const bool l_wins = ll > best;
    best = l_wins ? ll : best;
    code = l_wins ? 2u : code;
    const float hn = lane == t ? uu : best;  // column 0: H[i][0] = H[i-1][0] + g
    dw |= code << (2 * k);
    hb[k] = hn;
    L.upv = up;
    L.h = hn;
  }
  // this block's words: lane l's cells j = t - l in [1, m]
  const int tl = kTail ? min(t0 + kNwUnroll - 1, tend) : t0 + kNwUnroll - 1;
  if (rowok && tl >= lane + 1 && t0 <= lane + m) {
    const int64_t w = (int64_t)(i - 1) * Wr + ((t0 >> 4) - (lane >> 4));
    // the persistent-grid sweep's words are traced back by a wave that may
    // run on another CU: 8-byte {word, tag} entries, like its boundary rows
    if (kTagged)
      __hip_atomic_store((uint64_t *)dirs + w, ((uint64_t)pp.tag << 32) | dw, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    else
      dirs[w] = dw;
  }
  if (keep_row) {
    // lane k stores the last row's H at column t0 + k - lastlane
    float v = 0.0f;
#pragma unroll
    for (int k = 0; k < kNwUnroll; k++) {
      const float x = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hb[k]), lastlane));
      v = lane == k ? x : v;
    }
    const int j = t0 + lane - lastlane;
    if (lane < kNwUnroll && j >= 0 && j <= m && t0 + lane <= tl) {
      if (kTagged)
        __hip_atomic_store((uint64_t *)rowbuf + j, ((uint64_t)pp.tag << 32) | __float_as_uint(v), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      else
        rowbuf[j] = v;
    }
    if (!kTagged && pp.prog) {
      const int cols = min(m, tl - lastlane) + 1;
      if (cols > 0) nw_publish(pp, s, cols);
    }
  }
}

// One 64-row strip of a pair's sweep.  rowin: the previous strip's bottom
// row (strips after the first), rowout: this strip's bottom row (strips before
// the last; may be the same array as rowin for a one-wave sweep, whose reads
// run ahead of its writes); kTagged: rows of 8-byte {H, tag} entries (the
// persistent-grid sweep).  Returns H of the strip's last row at column m.
template <bool kTagged>
__device__ __forceinline__ float nw_strip(const NwArgs &a, const PairDesc &d, int s, uint32_t *dirs,
                                          const float *rowin, float *rowout, const NwPipe &pp) {
  const int lane = threadIdx.x & 63;
  const int n = d.n, m = d.m;
  const float g = a.gap;
  const int Wr = nw_dir_row_words(m);
  const int nstrips = (n + 63) >> 6;
  const int i = s * 64 + lane + 1;
  const bool rowok = i <= n;
  const int R = min(64, n - s * 64);
  const int lastlane = R - 1;
  const bool keep_row = s + 1 < nstrips;
  const float *blk = a.S + d.s_off + (int64_t)s * (m + 63) * 64;
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void *)blk, (short)0, (int)((m + R - 1) * R * 4), kBufferFlags);
  NwLane L{0.0f, 0.0f, -g, 0u};
  const int tend = m + lastlane;
  float bufA[kNwUnroll], bufB[kNwUnroll], rbA, rbB;
  int cd = -1;  // prefetch cursor: step t reads diagonal t-1
  const bool use_row = s > 0;
  // persistent-grid sweep: the first block's boundary-row entries, in flight
  uint64_t pend = 0;
  if (kTagged && use_row && lane < kNwUnroll && lane <= m)
    pend = __hip_atomic_load((const uint64_t *)rowin + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  nw_prefetch<kTagged>(bufA, rbA, rs, rowin, use_row, cd, lane, R, m, pp, s, pend);
  int t0 = 0;
  // full blocks of 2 x 16 steps
  for (; t0 + 2 * kNwUnroll - 1 <= tend; t0 += 2 * kNwUnroll) {
    nw_prefetch<kTagged>(bufB, rbB, rs, rowin, use_row, cd, lane, R, m, pp, s, pend);
    if (s == 0)
      nw_steps<false, true, kTagged>(bufA, rbA, t0, tend, L, lane, i, rowok, lastlane, keep_row, m, Wr, g, dirs, rowout, pp, s);
    else
      nw_steps<false, false, kTagged>(bufA, rbA, t0, tend, L, lane, i, rowok, lastlane, keep_row, m, Wr, g, dirs, rowout, pp, s);
    nw_prefetch<kTagged>(bufA, rbA, rs, rowin, use_row, cd, lane, R, m, pp, s, pend);
    if (s == 0)
      nw_steps<false, true, kTagged>(bufB, rbB, t0 + kNwUnroll, tend, L, lane, i, rowok, lastlane, keep_row, m, Wr, g, dirs,
                            rowout, pp, s);
    else
      nw_steps<false, false, kTagged>(bufB, rbB, t0 + kNwUnroll, tend, L, lane, i, rowok, lastlane, keep_row, m, Wr, g, dirs,
                             rowout, pp, s);
  }
  // the rest: at most two blocks, the last one partial
  for (; t0 <= tend; t0 += kNwUnroll) {
    if (s == 0)
      nw_steps<true, true, kTagged>(bufA, rbA, t0, tend, L, lane, i, rowok, lastlane, keep_row, m, Wr, g, dirs, rowout, pp, s);
    else
      nw_steps<true, false, kTagged>(bufA, rbA, t0, tend, L, lane, i, rowok, lastlane, keep_row, m, Wr, g, dirs, rowout, pp, s);
    if (t0 + kNwUnroll <= tend) nw_prefetch<kTagged>(bufA, rbA, rs, rowin, use_row, cd, lane, R, m, pp, s, pend);
  }
  return __shfl(L.h, lastlane);
}

// H[n][m] of a pair with no sentence on one side: the boundary alone.
__device__ __forceinline__ float nw_boundary_only(int n, int m, float g) {
  float h = 0.0f;
  for (int k = 0; k < n + m; k++) h = __fadd_rn(h, g);
  return h;
}

// Direction word widx of a pair swept by the persistent grid: its 8-byte
// {word, tag} entry, read again (bounded) until it carries this launch's tag;
// a give-up sets the pair's flag (per lane: callable from divergent code).
__device__ __forceinline__ uint32_t nw_tagged_word(const uint32_t *dirs, int64_t widx, const NwPipe &tp) {
  const uint64_t *e = (const uint64_t *)dirs + widx;
  uint64_t v = __hip_atomic_load(e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if ((uint32_t)(v >> 32) != tp.tag) {
    const uint64_t t0 = wall_clock64();
    while ((uint32_t)(v >> 32) != tp.tag && wall_clock64() - t0 <= tp.limit) {
      __builtin_amdgcn_s_sleep(1);
      v = __hip_atomic_load(e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if ((uint32_t)(v >> 32) != tp.tag) __hip_atomic_store(tp.gabort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return (uint32_t)v;
}

// Traceback, threshold filter and outputs of one pair (one wave), once the
// sweep has written all direction words (kTagged: 8-byte entries of the
// persistent-grid sweep, checked against tp.tag).
template <bool kLds, bool kTagged = false>
__device__ __forceinline__ void nw_finish(const NwArgs &a, const PairDesc &d, int64_t p, const uint32_t *dirs,
                                          float hnm, const NwPipe &tp = NwPipe{}) {
  const int lane = threadIdx.x & 63;
  const int n = d.n, m = d.m;
  const int Wr = nw_dir_row_words(m);
  const float *S = a.S + d.s_off;

  // traceback
  const int cap = min(n, m);
  const int64_t slot_end = d.out_off + cap;
  char *mv = a.moves ? a.moves + a.moves_off[p] : nullptr;
  int K = 0, T = 0;
  if (mv) {
    // with the move string (debug entry): lane 0, one move at a time
    if (lane == 0) {
      int i = n, j = m, k = 0, t = 0;
      int64_t cur = -1;
      uint32_t word = 0;
      while (i > 0 && j > 0) {
        const int l = (i - 1) & 63, st = j + l;  // the cell's lane and sweep step
        const int64_t widx = (int64_t)(i - 1) * Wr + ((st >> 4) - (l >> 4));
        if (widx != cur) {
          word = kLds ? dirs[widx] : kTagged ? nw_tagged_word(dirs, widx, tp) : ((const volatile uint32_t *)dirs)[widx];
          cur = widx;
        }
        const uint32_t code = (word >> (2 * (st & 15))) & 3u;
        char c;
        if (code == 0) {
          a.slot_src[slot_end - 1 - k] = i - 1;
          a.slot_tgt[slot_end - 1 - k] = j - 1;
          k++;
          i--;
          j--;
          c = 'D';
        } else if (code == 1) {
          i--;
          c = 'U';
        } else {
          j--;
          c = 'L';
        }
        mv[(n + m - 1) - t] = c;
        t++;
      }
      while (i > 0) {
        i--;
        mv[(n + m - 1) - t] = 'U';
        t++;
      }
      while (j > 0) {
        j--;
        mv[(n + m - 1) - t] = 'L';
        t++;
      }
      K = k;
      T = t;
    }
    K = __shfl(K, 0);
    T = __shfl(T, 0);
  } else {
    // Wave-uniform walk (scalar unit) over a window of direction words held
    // in registers: lane q holds the three words of row wr0 - q that end at
    // the word of column wj0 (the position where the window was loaded), so
    // the walk reads them with readlane and reloads only when it leaves the
    // window (64 rows up or about 32 columns left).  Inside a word a run of
    // L moves is skipped at once: the next cell that is not an L move is the
    // highest code below the current position that is not 2.  Lane (k mod 64)
    // keeps the k-th diagonal move; each full batch of 64 is stored at once.
    int i = n, j = m, k = 0;
    int vs = 0, vt = 0;
    int wr0 = -1;                        // window's first row (0-based), -1: no window
    uint32_t w0 = 0, w1 = 0, w2 = 0;     // this lane's words wlo, wlo + 1, wlo + 2 of row wr0 - lane
    int wlo = 0;                         // this lane's first word index
    auto load_window = [&]() {
      wr0 = i - 1;
      const int r = wr0 - lane;
      w0 = w1 = w2 = 0;
      wlo = 0;
      if (r >= 0) {
        const int l = r & 63;
        const int wj = ((j + l) >> 4) - (l >> 4);
        wlo = max(0, wj - 2);
        const uint32_t *row = dirs + (int64_t)r * Wr;
        if (kLds) {
          w0 = row[wlo];
          if (wlo + 1 < Wr) w1 = row[wlo + 1];
          if (wlo + 2 < Wr) w2 = row[wlo + 2];
        } else if (kTagged) {
          // only the words the sweep wrote (this row's cells lie in words
          // lo_w .. hi_w): the others are never read by the walk, and their
          // entries carry no tag of this launch
          // (the three loads are issued together; a word without this
          // launch's tag yet is read again on its own)
          const uint64_t *e = (const uint64_t *)dirs + (int64_t)r * Wr;
          const int lo_w = ((l + 1) >> 4) - (l >> 4), hi_w = ((l + m) >> 4) - (l >> 4);
          const bool k0 = wlo >= lo_w && wlo <= hi_w, k1 = wlo + 1 >= lo_w && wlo + 1 <= hi_w,
                     k2 = wlo + 2 >= lo_w && wlo + 2 <= hi_w;
          const uint64_t v0 = k0 ? __hip_atomic_load(e + wlo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
          const uint64_t v1 = k1 ? __hip_atomic_load(e + wlo + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
          const uint64_t v2 = k2 ? __hip_atomic_load(e + wlo + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
          w0 = (uint32_t)v0;
          w1 = (uint32_t)v1;
          w2 = (uint32_t)v2;
          if (k0 && (uint32_t)(v0 >> 32) != tp.tag) w0 = nw_tagged_word(dirs, (int64_t)r * Wr + wlo, tp);
          if (k1 && (uint32_t)(v1 >> 32) != tp.tag) w1 = nw_tagged_word(dirs, (int64_t)r * Wr + wlo + 1, tp);
          if (k2 && (uint32_t)(v2 >> 32) != tp.tag) w2 = nw_tagged_word(dirs, (int64_t)r * Wr + wlo + 2, tp);
        } else {
          const volatile uint32_t *vrow = row;
          w0 = vrow[wlo];
          if (wlo + 1 < Wr) w1 = vrow[wlo + 1];
          if (wlo + 2 < Wr) w2 = vrow[wlo + 2];
        }
      }
    };
    while (i > 0 && j > 0) {
      const int l = (i - 1) & 63, st = j + l;
      const int wi = (st >> 4) - (l >> 4);
      int q = wr0 - (i - 1);
      int d = wr0 < 0 || q > 63 ? -1 : wi - __builtin_amdgcn_readlane(wlo, q);
      if (d < 0) {
        load_window();
        q = 0;
        d = wi - __builtin_amdgcn_readlane(wlo, 0);
      }
      const uint32_t word = (uint32_t)__builtin_amdgcn_readlane((int)(d == 0 ? w0 : (d == 1 ? w1 : w2)), q);
      const int pos = st & 15;
      const uint32_t notL = ~(word >> 1) & 0x55555555u & (0xFFFFFFFFu >> (30 - 2 * pos));
      if (notL == 0) {  // L moves down to the word's first step
        j -= min(pos + 1, j);
        continue;
      }
      const int qb = (31 - __builtin_clz(notL)) >> 1;
      if (j - (pos - qb) < 1) {  // the L run reaches column 0 first
        j = 0;
        break;
      }
      j -= pos - qb;
      if (((word >> (2 * qb)) & 3u) == 0u) {
        if (lane == (k & 63)) {
          vs = i - 1;
          vt = j - 1;
        }
        k++;
        if ((k & 63) == 0) {
          const int64_t r = slot_end - k + 63 - lane;  // move k - 64 + lane
          a.slot_src[r] = vs;
          a.slot_tgt[r] = vt;
        }
        j--;
      }
      i--;
    }
    if (lane < (k & 63)) {
      const int64_t r = slot_end - 1 - ((k & ~63) + lane);
      a.slot_src[r] = vs;
      a.slot_tgt[r] = vt;
    }
    K = k;
    T = n + m - k;
  }
  wave_sync_mem();
  if (mv) {  // move the forward path from the tail of the region to its front
    const int off = n + m - T;
    for (int b = 0; b < T; b += 64) {
      const int kk = b + lane;
      const char c = kk < T ? mv[off + kk] : 0;
      __builtin_amdgcn_wave_barrier();
      if (kk < T) mv[kk] = c;
    }
  }

  // threshold filter and compaction, in path order
  int kept = 0;
  for (int b = 0; b < K; b += 64) {
    const int k = b + lane;
    int si = 0, ti = 0;
    float sv = 0.0f;
    bool keep = false;
    if (k < K) {
      const int64_t r = slot_end - K + k;
      si = a.slot_src[r];
      ti = a.slot_tgt[r];
      sv = S[score_pos(si, ti, n, m)];
      keep = sv >= a.tau;
    }
    const uint64_t bal = __ballot(keep);
    const int pos = kept + __popcll(bal & ((1ull << lane) - 1ull));
    if (keep) {
      a.slot_src[d.out_off + pos] = si;
      a.slot_tgt[d.out_off + pos] = ti;
      a.slot_score[d.out_off + pos] = sv;
    }
    kept += __popcll(bal);
  }
  if (lane == 0) {
    a.counts[p] = kept;
    a.align[a.pair_base + p] = hnm;
    if (a.n_moves) a.n_moves[a.pair_base + p] = T;
  }
}

// A pair swept by one wave, strip after strip.
template <bool kLds>
__device__ __forceinline__ void nw_pair(const NwArgs &a, const PairDesc &d, int64_t p, uint32_t *dirs,
                                        float *rowbuf) {
  float hnm = 0.0f;
  if (d.n > 0 && d.m > 0) {
    const int nstrips = (d.n + 63) >> 6;
    for (int s = 0; s < nstrips; s++) {
      hnm = nw_strip<false>(a, d, s, dirs, rowbuf, rowbuf, NwPipe{});
      wave_sync_mem();
    }
  } else {
    hnm = nw_boundary_only(d.n, d.m, a.gap);
  }
  nw_finish<kLds>(a, d, p, dirs, hnm);
}

// The arguments of gap penalty blockIdx.y of a launch that sweeps several.
__device__ __forceinline__ NwArgs nw_gap_view(const NwArgs &a0) {
  NwArgs a = a0;
  if (a.gaps) {
    const int64_t g = blockIdx.y;
    a.gap = a.gaps[g];
    a.dir_scratch += g * a.g_dirs;
    a.row_scratch += g * a.g_rows;
    a.slot_src += g * a.g_slots;
    a.slot_tgt += g * a.g_slots;
    a.slot_score += g * a.g_slots;
    a.counts += g * a.g_counts;
    a.align += g * a.g_align;
    a.ctrl += g * a.g_ctrl;
  }
  return a;
}

// A large pair whose sweep gave up: no accepted pairs, a NaN score, the
// call's status word set (lane 0).
__device__ __forceinline__ void nw_report_failed(const NwArgs &a, int64_t p) {
  a.counts[p] = 0;
  a.align[a.pair_base + p] = __int_as_float(0x7fc00000);
  if (a.n_moves) a.n_moves[a.pair_base + p] = 0;
  if (a.status) __hip_atomic_store(a.status, kStatusWaitGaveUp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// NPW pairs per workgroup, one wave each (waves never synchronise with each
// other).  Large pairs (nw_is_big) are left to nw_big_kernel.
template <int NPW>
__global__ __launch_bounds__(64 * NPW, 4) void nw_kernel(NwArgs a0) {
  const NwArgs a = nw_gap_view(a0);
  __shared__ uint32_t sdir_all[NPW][kDirLds];
  __shared__ float srow_all[NPW][kRowLds];
  const int wv = NPW == 1 ? 0 : __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t slot = (int64_t)blockIdx.x * NPW + wv;
  if (slot >= a.n_pairs) return;
  const int64_t p = a.order[slot];
  uint32_t *sdir = sdir_all[wv];
  float *srow = srow_all[wv];
  const PairDesc d = a.descs[p];
  if (nw_is_big(d.n)) return;
  if (d.dir_off < 0 && d.row_off < 0)
    nw_pair<true>(a, d, p, sdir, srow);
  else
    nw_pair<false>(a, d, p, d.dir_off < 0 ? sdir : a.dir_scratch + d.dir_off,
                   d.row_off < 0 ? srow : a.row_scratch + d.row_off);
}

// Large pairs: one workgroup of kNwBigWaves waves per pair.  Strip s is swept
// by wave s mod W; its lane 0 reads the bottom row of strip s - 1 as that
// strip publishes it (16 columns at a time, through global scratch with one
// row per strip boundary), so the strips run as a pipeline lagging about one
// block plus 64 steps behind each other.  Every wait is for a strip with a
// smaller index, swept by a wave of the same (co-resident) workgroup, so the
// pipeline always drains; each wait also ends after a time limit (default
// kNwWaitTicks), and the pair is then reported with no accepted pairs, a NaN
// score and the call's status word set, which the host turns into an error.
// After the sweep, wave 0 traces back.
__global__ __launch_bounds__(64 * kNwBigWaves) void nw_big_kernel(NwArgs a0) {
  const NwArgs a = nw_gap_view(a0);
  __shared__ int64_t prog[kNwBigWaves];
  __shared__ int abort_flag;
  __shared__ float s_hnm;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  for (int64_t bi = blockIdx.x; bi < a.n_big; bi += gridDim.x) {
    const int64_t p = a.big[bi];
    const PairDesc d = a.descs[p];
    if (threadIdx.x < kNwBigWaves) prog[threadIdx.x] = (int64_t)(-1ll * (1ll << 32));  // strip -1, 0 columns
    if (threadIdx.x == 0) {
      abort_flag = 0;
      s_hnm = 0.0f;
    }
    __syncthreads();
    uint32_t *dirs = a.dir_scratch + d.dir_off;
    float *rows = a.row_scratch + d.row_off;  // bottom row of strip s at rows + s (m + 1)
    const int nstrips = (d.n + 63) >> 6;
    const NwPipe pp{prog, kNwBigWaves, &abort_flag, a.wait_ticks};
    if (d.m <= 0) {  // no target sentence: the boundary alone
      if (threadIdx.x == 0) s_hnm = nw_boundary_only(d.n, d.m, a.gap);
    } else
    for (int s = wv; s < nstrips; s += kNwBigWaves) {
      const float h = nw_strip<false>(a, d, s, dirs, s > 0 ? rows + (int64_t)(s - 1) * (d.m + 1) : nullptr,
                               s + 1 < nstrips ? rows + (int64_t)s * (d.m + 1) : nullptr, pp);
      if (s == nstrips - 1 && lane == 0) s_hnm = h;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    if (wv == 0) {
      if (abort_flag) {  // the pair is reported as failed: NaN score, no pairs, status word set
        if (lane == 0) nw_report_failed(a, p);
      } else {
        nw_finish<false>(a, d, p, dirs, s_hnm);
      }
    }
    __syncthreads();
  }
}

// Large pairs with their strips spread over the whole GPU.  Every wave of a
// persistent grid takes tickets from a counter; the tickets are the strips of
// the large pairs, pair after pair (largest first) and in strip order inside
// a pair, so strip s - 1 was taken before strip s by a wave that is running
// or done, and a wait of strip s on it always ends (each wait is also
// bounded).  Everything one wave hands to another goes through global memory
// as 8-byte atomic entries {value, tag} that the reader reads again until
// they carry this launch's tag: the boundary rows (nw_row_take), the
// direction words and H[n][m].  No cache-wide fence is needed.  A wave that
// ends a strip counts it in its pair's control word; the wave that counts the
// last strip traces the pair back (or reports it failed).
__global__ __launch_bounds__(64 * kNwSplitWaves) void nw_split_kernel(NwArgs a0) {
  const NwArgs a = nw_gap_view(a0);
  const int lane = threadIdx.x & 63;
  int32_t *ctrl = a.ctrl;
  const uint32_t tag = (uint32_t)ctrl[1];
  for (;;) {
    int tk = 0;
    if (lane == 0) tk = __hip_atomic_fetch_add(ctrl, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    tk = __builtin_amdgcn_readfirstlane(tk);
    if (tk >= a.n_big_strips) break;
    const int bi = a.ticket_big[tk];
    const int s = tk - a.big_strip0[bi];
    const int64_t p = a.big[bi];
    const PairDesc d = a.descs[p];
    // {strips done, give-up flag, {H[n][m], tag} as one 8-byte entry}
    int32_t *pc = ctrl + kNwCtrlHead + (int64_t)kNwCtrlPerPair * bi;
    uint64_t *hslot = (uint64_t *)(pc + 2);
    const int nstrips = (d.n + 63) >> 6;
    uint32_t *dirs = a.dir_scratch + d.dir_off;
    float *rows = a.row_scratch + d.row_off;  // bottom row of strip s: 8-byte entries from rows + 2 s (m + 1)
    NwPipe pp;
    pp.limit = a.wait_ticks;
    pp.tag = tag;
    pp.gabort = pc + 1;
    float h = 0.0f;
    if (d.m > 0) {
      const int64_t rw = 2 * (int64_t)(d.m + 1);
      h = nw_strip<true>(a, d, s, dirs, s > 0 ? rows + (s - 1) * rw : nullptr, s + 1 < nstrips ? rows + s * rw : nullptr,
                         pp);
    } else {  // no target sentence: the boundary alone
      h = nw_boundary_only(d.n, d.m, a.gap);
    }
    if (s == nstrips - 1 && lane == 0)
      __hip_atomic_store(hslot, ((uint64_t)tag << 32) | __float_as_uint(h), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int done = 0;
    if (lane == 0) done = __hip_atomic_fetch_add(pc, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    done = __builtin_amdgcn_readfirstlane(done);
    if (done != nstrips - 1) continue;
    // the last strip of the pair: H[n][m] once its entry carries the tag, then the traceback
    float hnm = 0.0f;
    if (lane == 0) hnm = __uint_as_float(nw_tagged_word((const uint32_t *)hslot, 0, pp));
    hnm = __shfl(hnm, 0);
    if (__builtin_amdgcn_readfirstlane(__hip_atomic_load(pc + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == 0)
      nw_finish<false, true>(a, d, p, dirs, hnm, pp);
    // a give-up of any wait of the pair, the traceback's included: reported failed
    if (__builtin_amdgcn_readfirstlane(__hip_atomic_load(pc + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) &&
        lane == 0)
      nw_report_failed(a, p);
  }
}

// Tags of the persistent-grid NW launches on this device: each launch takes
// the next (never 0, so memory that was never written carries no valid tag).
__device__ uint32_t g_nw_tag;

// Control words of a persistent-grid NW launch (one workgroup): counters
// zeroed and the launch's new tag in every gap penalty's copy.
__global__ __launch_bounds__(256) void nw_split_begin_kernel(int32_t *ctrl, int64_t per_gap, int n_gaps) {
  __shared__ uint32_t tag;
  if (threadIdx.x == 0) {
    uint32_t t = atomicAdd(&g_nw_tag, 1u) + 1u;
    if (t == 0) t = atomicAdd(&g_nw_tag, 1u) + 1u;
    tag = t;
  }
  __syncthreads();
  for (int64_t k = threadIdx.x; k < per_gap * n_gaps; k += 256) ctrl[k] = (k % per_gap) == 1 ? (int32_t)tag : 0;
}

// ----------------------------------------------------------- compaction
__global__ __launch_bounds__(1024) void scan_kernel(const int32_t *counts, int64_t n, int64_t *po, int first) {
  __shared__ int64_t sh[16];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int64_t carry = first ? 0 : po[0];
  __syncthreads();
  if (first && tid == 0) po[0] = 0;
  for (int64_t base = 0; base < n; base += 4096) {
    int64_t v[4], s = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int64_t idx = base + tid * 4 + k;
      v[k] = idx < n ? counts[idx] : 0;
      s += v[k];
    }
    int64_t x = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == 63) sh[wv] = x;
    __syncthreads();
    int64_t wbase = 0, tot = 0;
    for (int w = 0; w < 16; w++) {
      wbase += w < wv ? sh[w] : 0;
      tot += sh[w];
    }
    int64_t run = carry + wbase + x - s;
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int64_t idx = base + tid * 4 + k;
      run += v[k];
      if (idx < n) po[idx + 1] = run;
    }
    carry += tot;
    __syncthreads();
  }
}

__global__ __launch_bounds__(64) void compact_kernel(const PairDesc *descs, int64_t n_pairs, const int32_t *counts,
                                                     const int64_t *po, const int32_t *slot_src,
                                                     const int32_t *slot_tgt, const float *slot_score,
                                                     int32_t *out_src, int32_t *out_tgt, float *out_score) {
  const int64_t p = blockIdx.x;
  if (p >= n_pairs) return;
  const int c = counts[p];
  const int64_t dst = po[p];
  const int64_t src = descs[p].out_off;
  for (int k = threadIdx.x; k < c; k += 64) {
    out_src[dst + k] = slot_src[src + k];
    out_tgt[dst + k] = slot_tgt[src + k];
    out_score[dst + k] = slot_score[src + k];
  }
}

// ---------------------------------------------------- tuning (NWT) counts
// For every accepted-before-threshold pair of every document pair (NW run
// with tau = -inf), and every threshold taus[t]: is it kept (score >= tau),
// and is it a reference pair?  Wave-level ballots feed two counters per t.
__global__ __launch_bounds__(64) void tune_count_kernel(const PairDesc *descs, int64_t n_pairs, int64_t pair_base,
                                                        const int32_t *counts, const int32_t *ssrc, const int32_t *stgt,
                                                        const float *sscore, const int64_t *truth_off,
                                                        const int32_t *truth_src, const int32_t *truth_tgt,
                                                        const float *taus, int n_taus,
                                                        unsigned long long *n_mined, unsigned long long *n_correct) {
  const int64_t p = blockIdx.x;
  if (p >= n_pairs) return;
  const int lane = threadIdx.x;
  const int c = counts[p];
  const int64_t base = descs[p].out_off;
  const int64_t t0 = truth_off[pair_base + p], t1 = truth_off[pair_base + p + 1];
  for (int k0 = 0; k0 < c; k0 += 64) {
    const int k = k0 + lane;
    const bool valid = k < c;
    int si = -1, ti = -1;
    float sv = 0.0f;
    bool hit = false;
    if (valid) {
      si = ssrc[base + k];
      ti = stgt[base + k];
      sv = sscore[base + k];
      for (int64_t e = t0; e < t1 && !hit; e++) hit = truth_src[e] == si && truth_tgt[e] == ti;
    }
    for (int t = 0; t < n_taus; t++) {
      const bool keep = valid && sv >= taus[t];
      const uint64_t bm = __ballot(keep), bc = __ballot(keep && hit);
      if (lane == 0) {
        if (bm) atomicAdd(&n_mined[t], (unsigned long long)__popcll(bm));
        if (bc) atomicAdd(&n_correct[t], (unsigned long long)__popcll(bc));
      }
    }
  }
}

// ---------------------------------------------- bidirectional union (BI)
// Pair p's forward result (i, j) and reverse result, mined with source and
// target swapped and mapped back to (i, j) = (its target index, its source
// index), are both strictly increasing in i and j; their union, without
// duplicates and ordered by (i, j), is merged by one lane per pair.  The
// forward score is kept for pairs found both ways.  Pass 1 counts, pass 2
// writes at the scanned offsets.
__global__ __launch_bounds__(64) void merge_bi_kernel(int64_t n_pairs, const int64_t *po_f, const int32_t *sf,
                                                      const int32_t *tf, const float *scf, const int64_t *po_r,
                                                      const int32_t *sr, const int32_t *tr, const float *scr,
                                                      int32_t *counts, const int64_t *po_out, int32_t *osrc,
                                                      int32_t *otgt, float *osc) {
  const int64_t p = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (p >= n_pairs) return;
  int64_t a = po_f[p], ae = po_f[p + 1], b = po_r[p], be = po_r[p + 1];
  int64_t o = po_out ? po_out[p] : 0;
  int k = 0;
  while (a < ae || b < be) {
    int i, j;
    float v;
    if (b >= be || (a < ae && (sf[a] < tr[b] || (sf[a] == tr[b] && tf[a] <= sr[b])))) {
      i = sf[a];
      j = tf[a];
      v = scf[a];
      if (b < be && tr[b] == i && sr[b] == j) b++;
      a++;
    } else {
      i = tr[b];
      j = sr[b];
      v = scr[b];
      b++;
    }
    if (po_out) {
      osrc[o + k] = i;
      otgt[o + k] = j;
      osc[o + k] = v;
    }
    k++;
  }
  if (!po_out) counts[p] = k;
}

__global__ void fill_i32_kernel(int32_t *p, int32_t v, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < n) p[k] = v;
}

// --------------------------------------------------------------- launches
hipError_t launch_lex_insert(const int32_t *keys, const int32_t *cnts, const int64_t *offs, const int32_t *vals,
                             int64_t n, int4 *slots, uint32_t mask, int shift, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(lex_insert_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, keys, cnts, offs, vals,
                     n, slots, mask, shift);
  return hipGetLastError();
}

hipError_t launch_lex_dense(const int32_t *keys, const int32_t *cnts, const int64_t *offs, const int32_t *vals, int64_t n,
                            int4 *dense, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(lex_dense_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, keys, cnts, offs, vals, n,
                     dense);
  return hipGetLastError();
}

hipError_t launch_translate(const int32_t *tok, int64_t n, const LexDev &L, int4 *out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(translate_kernel, dim3((unsigned)((n + 256 * kTransPerThread - 1) / (256 * kTransPerThread))),
                     dim3(256), 0, st, tok, n, L, out);
  return hipGetLastError();
}

hipError_t launch_score_table(float w0, float w1, float w2, float w3, float *table, hipStream_t st) {
  constexpr int N = kTabLen * kTabLen * kTabLen * kTabLen;
  hipLaunchKernelGGL(score_table_kernel, dim3(N / 256), dim3(256), 0, st, w0, w1, w2, w3, table);
  return hipGetLastError();
}

hipError_t launch_similarity(const SimArgs &a, int grid, int variant, hipStream_t st) {
  if (a.n_items <= 0) return hipSuccess;
  if (variant == 0)
    hipLaunchKernelGGL(sim_tile_kernel, dim3(grid), dim3(kTileThreads), 0, st, a);
  else if (variant == 3)
    hipLaunchKernelGGL(sim_bits_kernel<1280>, dim3(grid), dim3(kBitsThreads), 0, st, a);
  else if (variant == 4)
    hipLaunchKernelGGL(sim_bits_kernel<2048>, dim3(grid), dim3(kBitsThreads), 0, st, a);
  else if (variant == 2)
    hipLaunchKernelGGL(sim_kernel<true>, dim3(grid), dim3(kSimThreads), 0, st, a);
  else
    hipLaunchKernelGGL(sim_kernel<false>, dim3(grid), dim3(kSimThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_nw(const NwArgs &a, int pairs_per_group, hipStream_t st) {
  if (a.n_pairs <= 0) return hipSuccess;
  const unsigned G = a.gaps ? (unsigned)std::max(a.n_gaps, 1) : 1u;  // grid y: gap penalty
  if (a.n_big > 0 && a.split) {
    if (!a.ctrl || !a.big_strip0 || !a.ticket_big || a.n_big_strips <= 0) return hipErrorInvalidValue;
    const int64_t per_gap = kNwCtrlHead + (int64_t)kNwCtrlPerPair * a.n_big;
    if (G > 1 && a.g_ctrl != per_gap) return hipErrorInvalidValue;
    hipLaunchKernelGGL(nw_split_begin_kernel, dim3(1), dim3(256), 0, st, a.ctrl, per_gap, (int)G);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t groups = std::min<int64_t>((a.n_big_strips + kNwSplitWaves - 1) / kNwSplitWaves,
                                             (int64_t)kNwSplitGroupsPerCu * kNwSplitCus);
    hipLaunchKernelGGL(nw_split_kernel, dim3((unsigned)groups, G), dim3(64 * kNwSplitWaves), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  } else if (a.n_big > 0) {
    hipLaunchKernelGGL(nw_big_kernel, dim3((unsigned)std::min<int64_t>(a.n_big, 1024), G), dim3(64 * kNwBigWaves), 0,
                       st, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  switch (pairs_per_group) {
    case 1:
      hipLaunchKernelGGL(nw_kernel<1>, dim3((unsigned)a.n_pairs, G), dim3(64), 0, st, a);
      break;
    case 2:
      hipLaunchKernelGGL(nw_kernel<2>, dim3((unsigned)((a.n_pairs + 1) / 2), G), dim3(128), 0, st, a);
      break;
    case 4:
      hipLaunchKernelGGL(nw_kernel<4>, dim3((unsigned)((a.n_pairs + 3) / 4), G), dim3(256), 0, st, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_scan(const int32_t *counts, int64_t n, int64_t *po, int first, hipStream_t st) {
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, counts, n, po, first);
  return hipGetLastError();
}

hipError_t launch_compact(const PairDesc *descs, int64_t n_pairs, const int32_t *counts, const int64_t *po,
                          const int32_t *slot_src, const int32_t *slot_tgt, const float *slot_score, int32_t *out_src,
                          int32_t *out_tgt, float *out_score, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(compact_kernel, dim3((unsigned)n_pairs), dim3(64), 0, st, descs, n_pairs, counts, po, slot_src,
                     slot_tgt, slot_score, out_src, out_tgt, out_score);
  return hipGetLastError();
}

hipError_t launch_relayout(const PairDesc *descs, int64_t n_pairs, const float *src, float *dst, int to_diag,
                           hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(relayout_kernel, dim3(64, (unsigned)n_pairs), dim3(256), 0, st, descs, n_pairs, src, dst, to_diag);
  return hipGetLastError();
}

hipError_t launch_tune_count(const PairDesc *descs, int64_t n_pairs, int64_t pair_base, const int32_t *counts,
                             const int32_t *ssrc, const int32_t *stgt, const float *sscore, const int64_t *truth_off,
                             const int32_t *truth_src, const int32_t *truth_tgt, const float *taus, int n_taus,
                             unsigned long long *n_mined, unsigned long long *n_correct, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(tune_count_kernel, dim3((unsigned)n_pairs), dim3(64), 0, st, descs, n_pairs, pair_base, counts,
                     ssrc, stgt, sscore, truth_off, truth_src, truth_tgt, taus, n_taus, n_mined, n_correct);
  return hipGetLastError();
}

hipError_t launch_merge_bi(int64_t n_pairs, const int64_t *po_f, const int32_t *sf, const int32_t *tf, const float *scf,
                           const int64_t *po_r, const int32_t *sr, const int32_t *tr, const float *scr, int32_t *counts,
                           const int64_t *po_out, int32_t *osrc, int32_t *otgt, float *osc, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(merge_bi_kernel, dim3((unsigned)((n_pairs + 63) / 64)), dim3(64), 0, st, n_pairs, po_f, sf, tf, scf,
                     po_r, sr, tr, scr, counts, po_out, osrc, otgt, osc);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

}  // namespace ym
