// Device kernels of libymine for gfx950 (CDNA4, wave64).
//
//   lex_insert_kernel    builds the HBM-resident lexicon hash (session setup)
//   score_table_kernel   sentence-pair score for every (a, b, m_s, m_t) with
//                        a, b < 32, from the current classifier weights
//   sim_kernel           (a) sentence-pair score matrix of each document pair
//   nw_kernel            (b) Needleman-Wunsch forward pass, traceback and
//                        threshold filter of each document pair
//   scan_kernel,
//   compact_kernel       per-pair counts -> CSR offsets, slot -> CSR copy
//
// Floating point: the score is built from correctly rounded float divides,
// products and sums in a fixed order (no contraction; built with
// -ffp-contract=off and explicit __f*_rn), and the logistic is evaluated in
// double and rounded once.  The DP uses only float additions and strict
// comparisons.  Denormals are preserved.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ym_internal.h"

namespace ym {

__device__ __forceinline__ uint32_t hash32(int32_t x) { return (uint32_t)x * 0x9E3779B1u; }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ score
// Section 4: the classifier's confidence is a probability.  Features are the
// lexicon-overlap fractions f1 = m_s/a, f2 = m_t/b and the length ratio
// f3 = min/max; z = ((w0 + w1 f1) + w2 f2) + w3 f3; S = 1 / (1 + e^-z).
__device__ __forceinline__ float ratio_rn(int num, int den) {
  return den == 0 ? 0.0f : __fdiv_rn((float)num, (float)den);
}

__device__ float score_direct(float w0, float w1, float w2, float w3, int ms, int a, int mt, int b) {
  const float f1 = ratio_rn(ms, a);
  const float f2 = ratio_rn(mt, b);
  const float f3 = ratio_rn(a < b ? a : b, a < b ? b : a);
  float z = __fadd_rn(w0, __fmul_rn(w1, f1));
  z = __fadd_rn(z, __fmul_rn(w2, f2));
  z = __fadd_rn(z, __fmul_rn(w3, f3));
  const double e = exp(-(double)z);
  return (float)(1.0 / (1.0 + e));
}

__global__ __launch_bounds__(256) void score_table_kernel(float w0, float w1, float w2, float w3, float *table) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  const int mt = idx & 31, ms = (idx >> 5) & 31, b = (idx >> 10) & 31, a = (idx >> 15) & 31;
  table[idx] = score_direct(w0, w1, w2, w3, ms, a, mt, b);
}

// ---------------------------------------------------------------- lexicon
__global__ __launch_bounds__(256) void lex_insert_kernel(const int32_t *keys, const int32_t *cnts,
                                                         const int64_t *offs, int64_t n, int4 *slots,
                                                         uint32_t mask, int shift) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  const int32_t key = keys[k];
  uint32_t h = hash32(key) >> shift;
  for (;;) {  // load factor <= 1/2 and distinct keys: an empty slot is always reached
    const int prev = atomicCAS(&slots[h].x, kEmpty, key);
    if (prev == kEmpty) {
      slots[h].y = cnts[k];
      slots[h].z = (int32_t)offs[k];
      return;
    }
    h = (h + 1) & mask;
  }
}

// {offset, count} of T(x) in the value array; count 0 when x is not a key.
__device__ __forceinline__ int2 lex_find(const LexDev &L, int32_t x) {
  if (x < 0) return make_int2(0, 0);
  uint32_t h = hash32(x) >> L.shift;
  for (;;) {
    const int4 s = L.slots[h];
    if (s.x == x) return make_int2(s.z, s.y);
    if (s.x == kEmpty) return make_int2(0, 0);
    h = (h + 1) & L.mask;
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

// ------------------------------------------------------ (a) similarity
// One work item = (pair, source sentences [i0, i1)).  Target sentences are
// taken in chunks of at most kTcap tokens / kJcap sentences.  Each chunk's
// distinct target ids get dense local ids through an LDS hash, and the chunk's
// tokens are restaged in LDS as local ids.  A wave then owns one source
// sentence i at a time: it marks, in an LDS word per local id, which source
// positions q translate to that id (bit q) and whether the id is in X_i (top
// bit); every lane takes one target sentence j and walks its tokens:
//   m_t = number of tokens whose word has the top bit,
//   m_s = popcount of the OR of the words' position bits.
// Sentences longer than 31 tokens take one extra pass per further 31
// positions (position bits only).
__global__ __launch_bounds__(kSimThreads) void sim_kernel(SimArgs a) {
  __shared__ int32_t ukey[kUcap];
  __shared__ uint16_t ulid[kUcap];
  __shared__ uint16_t tdoc[kTcap];
  __shared__ uint16_t toff[kJcap + 1];
  __shared__ __align__(16) uint32_t Mw_all[kSimWaves][kTcap + 4];
  __shared__ int sh_scan[kSimWaves];
  __shared__ int sh_j1;

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  uint32_t *Mw = Mw_all[wv];

  for (int64_t item = blockIdx.x; item < a.n_items; item += gridDim.x) {
    const SimItem it = a.items[item];
    const PairDesc d = a.descs[it.pair];
    const int m = d.m;
    if (m <= 0 || it.i1 <= it.i0) continue;
    const int64_t *toffs = a.tgt_sent_off + d.tgt_sent0;
    const int64_t *soffs = a.src_sent_off + d.src_sent0;

    for (int j0 = 0; j0 < m;) {
      if (tid == 0) {
        const int64_t base = clamp64(toffs[j0], 0, a.n_tgt_tok);
        int lo = j0 + 1, hi = min(m, j0 + kJcap);
        while (lo < hi) {  // largest j1 whose tokens [j0, j1) fit kTcap (at least one sentence)
          const int mid = (lo + hi + 1) >> 1;
          if (clamp64(toffs[mid], 0, a.n_tgt_tok) - base <= kTcap)
            lo = mid;
          else
            hi = mid - 1;
        }
        sh_j1 = lo;
      }
      for (int s = tid; s < kUcap; s += kSimThreads) ukey[s] = kEmpty;
      __syncthreads();
      const int j1 = sh_j1;
      const int nj = j1 - j0;
      const int64_t tbase = clamp64(toffs[j0], 0, a.n_tgt_tok);
      const int ntok = (int)clamp64(clamp64(toffs[j1], 0, a.n_tgt_tok) - tbase, 0, kTcap);
      for (int jj = tid; jj <= nj; jj += kSimThreads)
        toff[jj] = (uint16_t)clamp64(clamp64(toffs[j0 + jj], 0, a.n_tgt_tok) - tbase, 0, ntok);
      for (int p = tid; p < ntok; p += kSimThreads) {
        const int32_t x = a.tgt_tok[tbase + p];
        tdoc[p] = x < 0 ? (uint16_t)0xFFFF : (uint16_t)u_insert(ukey, x);
      }
      __syncthreads();
      // dense local ids 1..nlid-1 in slot order (0 = "no such id", its word stays 0)
      constexpr int kSpt = kUcap / kSimThreads;
      int cnt = 0;
#pragma unroll
      for (int k = 0; k < kSpt; k++) cnt += (ukey[tid * kSpt + k] != kEmpty);
      int total;
      int r = block_excl_sum256(cnt, sh_scan, &total);
#pragma unroll
      for (int k = 0; k < kSpt; k++) {
        const int s = tid * kSpt + k;
        if (ukey[s] != kEmpty) ulid[s] = (uint16_t)(1 + r++);
      }
      const int nlid = total + 1;
      __syncthreads();
      for (int p = tid; p < ntok; p += kSimThreads) {
        const uint16_t s = tdoc[p];
        tdoc[p] = s == 0xFFFF ? (uint16_t)0 : ulid[s];
      }
      __syncthreads();

      const int nq4 = (nlid + 3) >> 2;
      for (int i = it.i0 + wv; i < it.i1; i += kSimWaves) {
        const int64_t sb = clamp64(soffs[i], 0, a.n_src_tok);
        const int64_t se = clamp64(soffs[i + 1], sb, a.n_src_tok);
        const int ai = (int)min<int64_t>(se - sb, 0x7fffffff);
        const int npass = ai <= kPosBits ? 1 : (ai + kPosBits - 1) / kPosBits;
        uint32_t ms_acc[kJpass], mt_acc[kJpass];
#pragma unroll
        for (int tp = 0; tp < kJpass; tp++) ms_acc[tp] = mt_acc[tp] = 0;

        for (int c = 0; c < npass; c++) {
          for (int k = lane; k < nq4; k += 64) reinterpret_cast<uint4 *>(Mw)[k] = make_uint4(0, 0, 0, 0);
          wave_sync();
          const int qlo = c == 0 ? 0 : kPosBits * c;
          const int qhi = c == 0 ? ai : min(ai, kPosBits * c + kPosBits);
          for (int q = qlo + lane; q < qhi; q += 64) {
            const int2 oc = lex_find(a.lex, a.src_tok[sb + q]);
            const int rel = q - kPosBits * c;
            const uint32_t bits = (c == 0 ? kHitBit : 0u) | (rel >= 0 && rel < kPosBits ? (1u << rel) : 0u);
            for (int e = 0; e < oc.y; e++) {
              const int s = u_find(ukey, a.lex.vals[oc.x + e]);
              if (s >= 0) atomicOr(&Mw[ulid[s]], bits);
            }
          }
          wave_sync();
#pragma unroll
          for (int tp = 0; tp < kJpass; tp++) {
            if (tp * 64 < nj) {
              const int jj = tp * 64 + lane;
              if (jj < nj) {
                const int p0 = toff[jj], p1 = toff[jj + 1];
                uint32_t acc = 0, mt = 0;
                for (int p = p0; p < p1; p++) {
                  const uint32_t mk = Mw[tdoc[p]];
                  mt += mk >> 31;
                  acc |= mk;
                }
                ms_acc[tp] += __popc(acc & ~kHitBit);
                if (c == 0) mt_acc[tp] = mt;
              }
            }
          }
          wave_sync();
        }
        float *Srow = a.S + d.s_off + (int64_t)i * m + j0;
#pragma unroll
        for (int tp = 0; tp < kJpass; tp++) {
          const int jj = tp * 64 + lane;
          if (tp * 64 < nj && jj < nj) {
            const int bj = toff[jj + 1] - toff[jj];
            const int ms = (int)ms_acc[tp], mt = (int)mt_acc[tp];
            const float sv = (ai < kTabLen && bj < kTabLen)
                                 ? a.table[((ai * kTabLen + bj) * kTabLen + ms) * kTabLen + mt]
                                 : score_direct(a.w0, a.w1, a.w2, a.w3, ms, ai, mt, bj);
            Srow[jj] = sv;
            if (a.ms_out) {
              const int64_t cell = d.s_off + (int64_t)i * m + j0 + jj;
              a.ms_out[cell] = ms;
              a.mt_out[cell] = mt;
            }
          }
        }
      }
      __syncthreads();
      j0 = j1;
    }
  }
}

// ------------------------------------------------------------- (b) NW
// One wave per document pair.  Rows are taken in strips of 64 (lane l owns
// DP row 64*s + l + 1); the strip sweeps the columns along anti-diagonals:
// at step t lane l computes column j = t - l.  The value from the row above
// arrives from lane l-1 through a one-lane DPP shift; lane 0 reads it from the
// previous strip's bottom row (or the top boundary, built by repeated
// addition).  Direction codes (D=0, U=1, L=2) are packed 16 per word, row-
// major, in LDS when the pair fits, else in global scratch.  Lane 0 then walks
// the path back from (n, m), writing the D cells backwards into the pair's
// output slots; the wave reads their scores, keeps those >= tau and compacts
// them in path order to the front of the slots.
__device__ __forceinline__ float shift_up_one_lane(float v) {
  // wave_shr:1 -- lane l receives lane l-1's value (lane 0 keeps its own)
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x138, 0xF, 0xF, false));
}

template <bool kLds>
__device__ __forceinline__ void nw_pair(const NwArgs &a, const PairDesc &d, int64_t p, uint32_t *dirs,
                                        float *rowbuf) {
  const int lane = threadIdx.x;
  const int n = d.n, m = d.m;
  const float g = a.gap;
  const int W = (m + 15) >> 4;
  const float *S = a.S + d.s_off;
  float hnm = 0.0f;

  if (n > 0 && m > 0) {
    const int nstrips = (n + 63) >> 6;
    for (int s = 0; s < nstrips; s++) {
      const int i = s * 64 + lane + 1;
      const bool rowok = i <= n;
      const int lastlane = min(63, n - s * 64 - 1);
      const float *Srow = S + (int64_t)(rowok ? i - 1 : 0) * m;
      float h = 0.0f, upv = 0.0f, topv = 0.0f;
      float snext = rowok ? Srow[0] : 0.0f;
      uint32_t dw = 0;
      const int tend = m + lastlane;
      for (int t = 0; t <= tend; t++) {
        float up = shift_up_one_lane(h);
        if (lane == 0) {
          if (s == 0) {
            topv = t == 0 ? 0.0f : __fadd_rn(topv, g);
            up = topv;
          } else if (t <= m) {
            up = rowbuf[t];
          }
        }
        const int j = t - lane;
        if (rowok && j >= 0 && j <= m) {
          float hn;
          if (j == 0) {
            hn = __fadd_rn(up, g);
          } else {
            const float sv = snext;
            if (j < m) snext = Srow[j];
            const float dd = __fadd_rn(upv, sv);
            const float uu = __fadd_rn(up, g);
            const float ll = __fadd_rn(h, g);
            float best = dd;
            uint32_t code = 0;
            if (uu > best) {
              best = uu;
              code = 1;
            }
            if (ll > best) {
              best = ll;
              code = 2;
            }
            hn = best;
            const int jc = j - 1;
            dw |= code << (2 * (jc & 15));
            if ((jc & 15) == 15 || j == m) {
              dirs[(int64_t)(i - 1) * W + (jc >> 4)] = dw;
              dw = 0;
            }
          }
          upv = up;
          h = hn;
          if (lane == lastlane && s + 1 < nstrips) rowbuf[j] = hn;
        }
      }
      if (s == nstrips - 1) hnm = __shfl(h, lastlane);
      if (kLds)
        wave_sync();
      else
        __threadfence();
      __builtin_amdgcn_wave_barrier();
    }
  } else {
    float h = 0.0f;
    for (int k = 0; k < n + m; k++) h = __fadd_rn(h, g);
    hnm = h;
  }

  // traceback (lane 0)
  const int cap = min(n, m);
  const int64_t slot_end = d.out_off + cap;
  char *mv = a.moves ? a.moves + a.moves_off[p] : nullptr;
  int K = 0, T = 0;
  if (lane == 0) {
    int i = n, j = m, k = 0, t = 0;
    int64_t cur = -1;
    uint32_t word = 0;
    while (i > 0 && j > 0) {
      const int jc = j - 1;
      const int64_t widx = (int64_t)(i - 1) * W + (jc >> 4);
      if (widx != cur) {
        word = dirs[widx];
        cur = widx;
      }
      const uint32_t code = (word >> (2 * (jc & 15))) & 3u;
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
      if (mv) mv[(n + m - 1) - t] = c;
      t++;
    }
    while (i > 0) {
      i--;
      if (mv) mv[(n + m - 1) - t] = 'U';
      t++;
    }
    while (j > 0) {
      j--;
      if (mv) mv[(n + m - 1) - t] = 'L';
      t++;
    }
    K = k;
    T = t;
  }
  K = __shfl(K, 0);
  T = __shfl(T, 0);
  __threadfence();
  __builtin_amdgcn_wave_barrier();
  if (mv) {  // move the forward path from the tail of the region to its front
    const int off = n + m - T;
    for (int b = 0; b < T; b += 64) {
      const int k = b + lane;
      const char c = k < T ? mv[off + k] : 0;
      __builtin_amdgcn_wave_barrier();
      if (k < T) mv[k] = c;
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
      sv = S[(int64_t)si * m + ti];
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

__global__ __launch_bounds__(64) void nw_kernel(NwArgs a) {
  __shared__ uint32_t sdir[kDirLds];
  __shared__ float srow[kRowLds];
  const int64_t p = blockIdx.x;
  if (p >= a.n_pairs) return;
  const PairDesc d = a.descs[p];
  if (d.dir_off < 0 && d.row_off < 0)
    nw_pair<true>(a, d, p, sdir, srow);
  else
    nw_pair<false>(a, d, p, d.dir_off < 0 ? sdir : a.dir_scratch + d.dir_off,
                   d.row_off < 0 ? srow : a.row_scratch + d.row_off);
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

__global__ void fill_i32_kernel(int32_t *p, int32_t v, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < n) p[k] = v;
}

// --------------------------------------------------------------- launches
hipError_t launch_lex_insert(const int32_t *keys, const int32_t *cnts, const int64_t *offs, int64_t n, int4 *slots,
                             uint32_t mask, int shift, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(lex_insert_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, keys, cnts, offs, n,
                     slots, mask, shift);
  return hipGetLastError();
}

hipError_t launch_score_table(float w0, float w1, float w2, float w3, float *table, hipStream_t st) {
  constexpr int N = kTabLen * kTabLen * kTabLen * kTabLen;
  hipLaunchKernelGGL(score_table_kernel, dim3(N / 256), dim3(256), 0, st, w0, w1, w2, w3, table);
  return hipGetLastError();
}

hipError_t launch_similarity(const SimArgs &a, int grid, hipStream_t st) {
  if (a.n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(sim_kernel, dim3(grid), dim3(kSimThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_nw(const NwArgs &a, hipStream_t st) {
  if (a.n_pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(nw_kernel, dim3((unsigned)a.n_pairs), dim3(64), 0, st, a);
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

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

}  // namespace ym
