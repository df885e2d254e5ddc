/*
 * Seeded synthetic comparable-corpus generator.
 *
 * The paper mines 1,000 comparable Wikipedia article pairs (Table 3) and the
 * corpora of Table 1; none of them is available here, so both the GPU miner
 * and the CPU oracle are fed documents drawn by this generator instead.  It
 * holds none of the method's arithmetic: it only draws token ids, sentence
 * lengths and counts, a bilingual lexicon, classifier weights and arrival
 * times.  Both sides receive its output as plain arrays.
 *
 * Randomness is counter based so that any pair can be regenerated alone:
 * value k of the stream (seed, pair, purpose) is SplitMix64's output mix
 * applied to key + k * golden-gamma, where key is derived from the triple by
 * the same mix (Steele, Lea & Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014).
 *
 * Workload shape (per document pair):
 *   - n source and m target sentence counts from a fixed value, a uniform
 *     range, or a capped lognormal;
 *   - sentence lengths uniform in [len_min, len_max], token ids Zipf(s) over a
 *     vocabulary of V ids (rank r -> id r-1), inverse-CDF sampled;
 *   - a fraction of source sentences is "planted": the target document holds
 *     a noisy lexicon translation of each (every token replaced with
 *     probability replace_p by a uniform id, then +-indel_max insertions or
 *     deletions), kept in source order (optionally shuffled inside blocks) and
 *     interleaved at random positions among independent target sentences.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GAMMA 0x9e3779b97f4a7c15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

typedef struct {
  uint64_t key;
  uint64_t ctr;
} rng_t;

static rng_t rng_make(uint64_t seed, uint64_t a, uint64_t b) {
  rng_t r;
  r.key = mix64(mix64(seed * GAMMA + 0x632be59bd9b4e019ULL) ^ mix64(a + 0x8cb92ba72f3d8dd7ULL) ^
                mix64(b * 0xd1b54a32d192ed03ULL + 1));
  r.ctr = 0;
  return r;
}

static inline uint64_t rng_u64(rng_t *r) {
  r->ctr++;
  return mix64(r->key + r->ctr * GAMMA);
}

/* uniform double in [0, 1) with 53 random bits */
static inline double rng_unif(rng_t *r) { return (double)(rng_u64(r) >> 11) * 0x1.0p-53; }

/* uniform integer in [lo, hi] (inclusive); bias below 2^-40 for our ranges */
static inline int64_t rng_int(rng_t *r, int64_t lo, int64_t hi) {
  uint64_t span = (uint64_t)(hi - lo) + 1;
  return lo + (int64_t)(rng_u64(r) % span);
}

static inline double rng_normal(rng_t *r) {
  double u1 = rng_unif(r), u2 = rng_unif(r);
  if (u1 < 0x1.0p-60) u1 = 0x1.0p-60;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* ------------------------------------------------------------------ Zipf */
typedef struct {
  int32_t V;
  double s;
  double *cdf;     /* cdf[r-1] = P(rank <= r) */
  int32_t *guide;  /* guide[k]: smallest index with cdf > k / G (G a power of two) */
  int32_t lg;      /* G = 2^lg */
} zipf_t;

static int zipf_init(zipf_t *z, int32_t V, double s) {
  z->V = V;
  z->s = s;
  z->cdf = (double *)malloc(sizeof(double) * (size_t)V);
  if (!z->cdf) return -1;
  double acc = 0.0;
  for (int32_t r = 1; r <= V; r++) {
    acc += pow((double)r, -s);
    z->cdf[r - 1] = acc;
  }
  for (int32_t r = 0; r < V; r++) z->cdf[r] /= acc;
  z->cdf[V - 1] = 1.0;
  /* guide table of the inverse CDF (about four buckets per rank, at most 2^22) */
  z->lg = 10;
  while (z->lg < 22 && ((int64_t)1 << z->lg) < 4 * (int64_t)V) z->lg++;
  const int64_t G = (int64_t)1 << z->lg;
  z->guide = (int32_t *)malloc(sizeof(int32_t) * (size_t)G);
  if (!z->guide) {
    free(z->cdf);
    return -1;
  }
  int32_t r = 0;
  for (int64_t k = 0; k < G; k++) {
    const double t = (double)k / (double)G; /* exact: G is a power of two */
    while (r < V - 1 && z->cdf[r] <= t) r++;
    z->guide[k] = r;
  }
  return 0;
}

static void zipf_free(zipf_t *z) {
  free(z->cdf);
  free(z->guide);
  z->cdf = NULL;
  z->guide = NULL;
}

/* The smallest index r with cdf[r] > u (inverse-CDF sampling).  u * G is
 * exact, so every index below guide[floor(u G)] has cdf <= floor(u G) / G <= u
 * and the scan from there finds the same index as a binary search would. */
static inline int32_t zipf_draw(const zipf_t *z, rng_t *r) {
  const double u = rng_unif(r);
  int32_t k = z->guide[(int64_t)(u * (double)((int64_t)1 << z->lg))];
  while (k < z->V - 1 && z->cdf[k] <= u) k++;
  return k;
}

/* ------------------------------------------------------------ config */
typedef struct {
  int32_t vocab;
  double zipf_s;
  int32_t len_min, len_max;
  int32_t count_kind; /* 0 fixed, 1 uniform, 2 lognormal */
  int32_t n_fixed, m_fixed;
  int32_t cmin, cmax;
  double ln_median, ln_sigma;
  int32_t ln_cap;
  double plant_frac;
  double replace_p;
  int32_t indel_max;
  int32_t shuffle_block;     /* 0: planted targets keep source order */
  int32_t primary_only;      /* 1: translate with the first listed target id */
} synth_cfg;

/* purposes of the per-pair streams */
enum { P_SIZES = 1, P_SRC = 2, P_PICK = 3, P_NOISE = 4, P_INDEP = 5, P_PLACE = 6, P_SHUF = 7 };

/* growable int buffers */
typedef struct {
  int64_t *p;
  int64_t n, cap;
} vec64;
typedef struct {
  int32_t *p;
  int64_t n, cap;
} vec32;

static int v64_push(vec64 *v, int64_t x) {
  if (v->n == v->cap) {
    int64_t c = v->cap ? v->cap * 2 : 1024;
    int64_t *q = (int64_t *)realloc(v->p, sizeof(int64_t) * (size_t)c);
    if (!q) return -1;
    v->p = q;
    v->cap = c;
  }
  v->p[v->n++] = x;
  return 0;
}
static int v32_push(vec32 *v, int32_t x) {
  if (v->n == v->cap) {
    int64_t c = v->cap ? v->cap * 2 : 4096;
    int32_t *q = (int32_t *)realloc(v->p, sizeof(int32_t) * (size_t)c);
    if (!q) return -1;
    v->p = q;
    v->cap = c;
  }
  v->p[v->n++] = x;
  return 0;
}

/* Output of synth_generate: malloc'ed arrays, released by synth_free. */
typedef struct {
  int64_t n_pairs;
  int64_t *src_doc_off; /* n_pairs+1, sentence index */
  int64_t *src_sent_off; /* n_src_sent+1, token index */
  int32_t *src_tok;
  int64_t *tgt_doc_off;
  int64_t *tgt_sent_off;
  int32_t *tgt_tok;
  int64_t n_src_sent, n_tgt_sent, n_src_tok, n_tgt_tok;
  int64_t *truth_off; /* n_pairs+1 */
  int32_t *truth_src, *truth_tgt;
  int64_t n_truth;
} synth_corpus;

static int32_t draw_count(const synth_cfg *c, rng_t *r, int side) {
  switch (c->count_kind) {
    case 0:
      return side ? c->m_fixed : c->n_fixed;
    case 1:
      return (int32_t)rng_int(r, c->cmin, c->cmax);
    default: {
      double v = exp(log(c->ln_median) + c->ln_sigma * rng_normal(r));
      double rv = floor(v + 0.5);
      if (rv < 1.0) rv = 1.0;
      if (rv > (double)c->ln_cap) rv = (double)c->ln_cap;
      return (int32_t)rv;
    }
  }
}

typedef struct {
  /* translation lookup by source id < V: first/count into lex_tgt */
  const int64_t *first;
  const int32_t *count;
  const int32_t *tgt;
} lexview;

static int append_sentence_zipf(const synth_cfg *c, const zipf_t *z, rng_t *r, vec32 *tok, vec64 *sent) {
  int32_t len = (int32_t)rng_int(r, c->len_min, c->len_max);
  for (int32_t k = 0; k < len; k++)
    if (v32_push(tok, zipf_draw(z, r))) return -1;
  return v64_push(sent, tok->n);
}

int synth_free(synth_corpus *o) {
  if (!o) return 0;
  free(o->src_doc_off);
  free(o->src_sent_off);
  free(o->src_tok);
  free(o->tgt_doc_off);
  free(o->tgt_sent_off);
  free(o->tgt_tok);
  free(o->truth_off);
  free(o->truth_src);
  free(o->truth_tgt);
  memset(o, 0, sizeof(*o));
  return 0;
}

/*
 * Generate pairs pair_ids[0..n_pairs) of the corpus (cfg, seed).  Each pair
 * depends only on (cfg, seed, its id, lexicon), so a subset is reproduced
 * exactly by listing its ids.
 * Lexicon is CSR over source ids: lex_first/lex_count indexed by id < V.
 */
static int generate_serial(const synth_cfg *c, const zipf_t *zp, uint64_t seed, const int64_t *pair_ids,
                           int64_t n_pairs, const int64_t *lex_first, const int32_t *lex_count,
                           const int32_t *lex_tgt, synth_corpus *out) {
  memset(out, 0, sizeof(*out));
  const zipf_t z = *zp;
  lexview lx = {lex_first, lex_count, lex_tgt};

  vec64 sdoc = {0}, tdoc = {0}, ssent = {0}, tsent = {0}, toff = {0};
  vec32 stok = {0}, ttok = {0}, trs = {0}, trt = {0};
  int rc = 0;
  /* scratch for one pair */
  int32_t *pick = NULL, *order = NULL, *place = NULL, *buf = NULL;
  int64_t cap_n = 0;
  char *is_plant = NULL;
  int64_t cap_m = 0;
  int64_t *ind_sent = NULL; /* temp target sentence boundaries */
  vec32 planted_tok = {0}, indep_tok = {0};
  vec64 planted_off = {0}, indep_off = {0};

  rc |= v64_push(&sdoc, 0);
  rc |= v64_push(&tdoc, 0);
  rc |= v64_push(&ssent, 0);
  rc |= v64_push(&tsent, 0);
  rc |= v64_push(&toff, 0);
  if (rc) goto fail;

  for (int64_t pi = 0; pi < n_pairs; pi++) {
    int64_t pid = pair_ids[pi];
    rng_t rs = rng_make(seed, (uint64_t)pid, P_SIZES);
    int32_t n = draw_count(c, &rs, 0);
    int32_t m = draw_count(c, &rs, 1);
    if (n > cap_n || m > cap_n) {
      cap_n = (n > m ? n : m) + 16;
      free(pick);
      free(order);
      free(place);
      pick = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap_n);
      order = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap_n);
      place = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap_n);
      if (!pick || !order || !place) goto fail;
    }
    if (m > cap_m) {
      cap_m = m + 16;
      free(is_plant);
      is_plant = (char *)malloc((size_t)cap_m);
      if (!is_plant) goto fail;
    }

    /* source document */
    int64_t src_sent0 = ssent.n - 1;
    rng_t rsrc = rng_make(seed, (uint64_t)pid, P_SRC);
    for (int32_t i = 0; i < n; i++)
      if (append_sentence_zipf(c, &z, &rsrc, &stok, &ssent)) goto fail;

    /* which source sentences are planted: partial Fisher-Yates */
    int64_t P = (int64_t)floor(c->plant_frac * (double)n + 0.5);
    if (P > m) P = m;
    if (P > n) P = n;
    rng_t rpick = rng_make(seed, (uint64_t)pid, P_PICK);
    for (int32_t i = 0; i < n; i++) pick[i] = i;
    for (int64_t k = 0; k < P; k++) {
      int64_t j = rng_int(&rpick, k, n - 1);
      int32_t t = pick[k];
      pick[k] = pick[j];
      pick[j] = t;
    }
    /* sort chosen indices (insertion sort on small P is fine; use qsort-free merge) */
    for (int64_t a = 1; a < P; a++) {
      int32_t v = pick[a];
      int64_t b = a - 1;
      while (b >= 0 && pick[b] > v) {
        pick[b + 1] = pick[b];
        b--;
      }
      pick[b + 1] = v;
    }

    /* planted target sentences, in source order */
    planted_tok.n = 0;
    planted_off.n = 0;
    if (v64_push(&planted_off, 0)) goto fail;
    rng_t rnoise = rng_make(seed, (uint64_t)pid, P_NOISE);
    for (int64_t k = 0; k < P; k++) {
      int32_t si = pick[k];
      int64_t b0 = ssent.p[src_sent0 + si], b1 = ssent.p[src_sent0 + si + 1];
      int64_t start = planted_tok.n;
      for (int64_t q = b0; q < b1; q++) {
        int32_t x = stok.p[q];
        int32_t y;
        if (x < c->vocab && lx.count[x] > 0) {
          int32_t pickk = c->primary_only ? 0 : (int32_t)rng_int(&rnoise, 0, lx.count[x] - 1);
          y = lx.tgt[lx.first[x] + pickk];
        } else {
          y = (int32_t)rng_int(&rnoise, 0, c->vocab - 1);
        }
        if (c->replace_p > 0.0 && rng_unif(&rnoise) < c->replace_p)
          y = (int32_t)rng_int(&rnoise, 0, c->vocab - 1);
        if (v32_push(&planted_tok, y)) goto fail;
      }
      if (c->indel_max > 0) {
        int32_t kk = (int32_t)rng_int(&rnoise, -c->indel_max, c->indel_max);
        if (kk > 0) {
          for (int32_t e = 0; e < kk; e++) {
            int64_t len = planted_tok.n - start;
            int64_t pos = start + rng_int(&rnoise, 0, len);
            int32_t y = (int32_t)rng_int(&rnoise, 0, c->vocab - 1);
            if (v32_push(&planted_tok, 0)) goto fail;
            memmove(&planted_tok.p[pos + 1], &planted_tok.p[pos],
                    sizeof(int32_t) * (size_t)(planted_tok.n - 1 - pos));
            planted_tok.p[pos] = y;
          }
        } else if (kk < 0) {
          for (int32_t e = 0; e < -kk; e++) {
            int64_t len = planted_tok.n - start;
            if (len <= 1) break;
            int64_t pos = start + rng_int(&rnoise, 0, len - 1);
            memmove(&planted_tok.p[pos], &planted_tok.p[pos + 1],
                    sizeof(int32_t) * (size_t)(planted_tok.n - 1 - pos));
            planted_tok.n--;
          }
        }
      }
      if (v64_push(&planted_off, planted_tok.n)) goto fail;
    }

    /* independent target sentences */
    indep_tok.n = 0;
    indep_off.n = 0;
    if (v64_push(&indep_off, 0)) goto fail;
    rng_t rind = rng_make(seed, (uint64_t)pid, P_INDEP);
    for (int64_t k = 0; k < (int64_t)m - P; k++)
      if (append_sentence_zipf(c, &z, &rind, &indep_tok, &indep_off)) goto fail;

    /* order of planted items (identity, or shuffled inside blocks) */
    for (int64_t k = 0; k < P; k++) order[k] = (int32_t)k;
    if (c->shuffle_block > 1) {
      rng_t rsh = rng_make(seed, (uint64_t)pid, P_SHUF);
      for (int64_t b0 = 0; b0 < P; b0 += c->shuffle_block) {
        int64_t b1 = b0 + c->shuffle_block;
        if (b1 > P) b1 = P;
        for (int64_t k = b1 - 1; k > b0; k--) {
          int64_t j = rng_int(&rsh, b0, k);
          int32_t t = order[k];
          order[k] = order[j];
          order[j] = t;
        }
      }
    }

    /* positions of planted items among the m target slots */
    rng_t rpl = rng_make(seed, (uint64_t)pid, P_PLACE);
    for (int32_t j = 0; j < m; j++) place[j] = j;
    for (int64_t k = 0; k < P; k++) {
      int64_t j = rng_int(&rpl, k, m - 1);
      int32_t t = place[k];
      place[k] = place[j];
      place[j] = t;
    }
    memset(is_plant, 0, (size_t)m);
    for (int64_t k = 0; k < P; k++) is_plant[place[k]] = 1;

    /* assemble target document */
    int64_t kp = 0, ki = 0;
    for (int32_t j = 0; j < m; j++) {
      if (is_plant[j]) {
        int32_t item = order[kp++];
        for (int64_t q = planted_off.p[item]; q < planted_off.p[item + 1]; q++)
          if (v32_push(&ttok, planted_tok.p[q])) goto fail;
        if (v32_push(&trs, pick[item]) || v32_push(&trt, j)) goto fail;
      } else {
        for (int64_t q = indep_off.p[ki]; q < indep_off.p[ki + 1]; q++)
          if (v32_push(&ttok, indep_tok.p[q])) goto fail;
        ki++;
      }
      if (v64_push(&tsent, ttok.n)) goto fail;
    }
    if (v64_push(&sdoc, ssent.n - 1) || v64_push(&tdoc, tsent.n - 1) || v64_push(&toff, trs.n))
      goto fail;
  }

  out->n_pairs = n_pairs;
  out->src_doc_off = sdoc.p;
  out->tgt_doc_off = tdoc.p;
  out->src_sent_off = ssent.p;
  out->tgt_sent_off = tsent.p;
  out->src_tok = stok.p;
  out->tgt_tok = ttok.p;
  out->n_src_sent = ssent.n - 1;
  out->n_tgt_sent = tsent.n - 1;
  out->n_src_tok = stok.n;
  out->n_tgt_tok = ttok.n;
  out->truth_off = toff.p;
  out->truth_src = trs.p;
  out->truth_tgt = trt.p;
  out->n_truth = trs.n;
  free(pick);
  free(order);
  free(place);
  free(is_plant);
  free(ind_sent);
  free(planted_tok.p);
  free(planted_off.p);
  free(indep_tok.p);
  free(indep_off.p);
  return 0;

fail:
  free(pick);
  free(order);
  free(place);
  free(is_plant);
  free(ind_sent);
  free(planted_tok.p);
  free(planted_off.p);
  free(indep_tok.p);
  free(indep_off.p);
  free(sdoc.p);
  free(tdoc.p);
  free(ssent.p);
  free(tsent.p);
  free(stok.p);
  free(ttok.p);
  free(toff.p);
  free(trs.p);
  free(trt.p);
  memset(out, 0, sizeof(*out));
  return -1;
}

int synth_generate(const synth_cfg *c, uint64_t seed, const int64_t *pair_ids, int64_t n_pairs,
                   const int64_t *lex_first, const int32_t *lex_count, const int32_t *lex_tgt,
                   synth_corpus *out) {
  memset(out, 0, sizeof(*out));
  zipf_t z;
  if (c->vocab <= 0 || c->len_min < 0 || c->len_max < c->len_min) return -2;
  if (zipf_init(&z, c->vocab, c->zipf_s)) return -1;
  const int rc = generate_serial(c, &z, seed, pair_ids, n_pairs, lex_first, lex_count, lex_tgt, out);
  zipf_free(&z);
  return rc;
}

/*
 * The same corpus generated by several threads, each over a contiguous range
 * of the listed pairs (every pair depends only on its own id, so the result is
 * identical).  synth_generate_mt leaves the parts in a job and reports the
 * totals; the caller allocates the output arrays and synth_collect copies the
 * parts into them (rebasing offsets) and releases the job.
 */
typedef struct {
  const synth_cfg *c;
  const zipf_t *z;
  uint64_t seed;
  const int64_t *ids;
  int64_t n;
  const int64_t *first;
  const int32_t *count;
  const int32_t *tgt;
  synth_corpus out;
  int rc;
} gen_part;

typedef struct {
  int n_parts;
  gen_part *parts;
} synth_job;

static void *gen_part_run(void *arg) {
  gen_part *g = (gen_part *)arg;
  g->rc = generate_serial(g->c, g->z, g->seed, g->ids, g->n, g->first, g->count, g->tgt, &g->out);
  return NULL;
}

static void job_free(synth_job *j) {
  if (!j) return;
  for (int k = 0; k < j->n_parts; k++) synth_free(&j->parts[k].out);
  free(j->parts);
  free(j);
}

/* totals[0..4]: source sentences, target sentences, source tokens, target
 * tokens, planted pairs */
int synth_generate_mt(const synth_cfg *c, uint64_t seed, const int64_t *pair_ids, int64_t n_pairs,
                      const int64_t *lex_first, const int32_t *lex_count, const int32_t *lex_tgt, int threads,
                      void **job_out, int64_t totals[5]) {
  *job_out = NULL;
  if (c->vocab <= 0 || c->len_min < 0 || c->len_max < c->len_min) return -2;
  zipf_t z;
  if (zipf_init(&z, c->vocab, c->zipf_s)) return -1;
  int T = threads < 1 ? 1 : threads;
  if ((int64_t)T > n_pairs / 16) T = n_pairs / 16 > 0 ? (int)(n_pairs / 16) : 1;
  synth_job *j = (synth_job *)calloc(1, sizeof(synth_job));
  gen_part *parts = j ? (gen_part *)calloc((size_t)T, sizeof(gen_part)) : NULL;
  pthread_t *th = (pthread_t *)calloc((size_t)T, sizeof(pthread_t));
  if (!j || !parts || !th) {
    free(j);
    free(parts);
    free(th);
    zipf_free(&z);
    return -1;
  }
  j->n_parts = T;
  j->parts = parts;
  int rc = 0;
  for (int k = 0; k < T; k++) {
    const int64_t p0 = n_pairs * k / T, p1 = n_pairs * (k + 1) / T;
    gen_part g = {c, &z, seed, pair_ids + p0, p1 - p0, lex_first, lex_count, lex_tgt, {0}, 0};
    parts[k] = g;
  }
  int started = 0;
  for (int k = 1; k < T; k++) {
    if (pthread_create(&th[k], NULL, gen_part_run, &parts[k]) != 0) {
      gen_part_run(&parts[k]);
      th[k] = 0;
    } else {
      started |= 1;
    }
  }
  gen_part_run(&parts[0]);
  for (int k = 1; k < T; k++)
    if (th[k]) pthread_join(th[k], NULL);
  (void)started;
  free(th);
  zipf_free(&z);
  for (int k = 0; k < T; k++) rc |= parts[k].rc;
  if (rc) {
    job_free(j);
    return -1;
  }
  for (int q = 0; q < 5; q++) totals[q] = 0;
  for (int k = 0; k < T; k++) {
    totals[0] += parts[k].out.n_src_sent;
    totals[1] += parts[k].out.n_tgt_sent;
    totals[2] += parts[k].out.n_src_tok;
    totals[3] += parts[k].out.n_tgt_tok;
    totals[4] += parts[k].out.n_truth;
  }
  *job_out = j;
  return 0;
}

typedef struct {
  const synth_corpus *in;
  int64_t pair0, ssent0, tsent0, stok0, ttok0, truth0;
  int64_t *sdoc, *ssent, *tdoc, *tsent, *toff;
  int32_t *stok, *ttok, *trs, *trt;
} collect_part;

static void *collect_run(void *arg) {
  collect_part *q = (collect_part *)arg;
  const synth_corpus *o = q->in;
  for (int64_t p = 1; p <= o->n_pairs; p++) {
    q->sdoc[q->pair0 + p] = q->ssent0 + o->src_doc_off[p];
    q->tdoc[q->pair0 + p] = q->tsent0 + o->tgt_doc_off[p];
    q->toff[q->pair0 + p] = q->truth0 + o->truth_off[p];
  }
  for (int64_t s = 1; s <= o->n_src_sent; s++) q->ssent[q->ssent0 + s] = q->stok0 + o->src_sent_off[s];
  for (int64_t s = 1; s <= o->n_tgt_sent; s++) q->tsent[q->tsent0 + s] = q->ttok0 + o->tgt_sent_off[s];
  if (o->n_src_tok) memcpy(q->stok + q->stok0, o->src_tok, sizeof(int32_t) * (size_t)o->n_src_tok);
  if (o->n_tgt_tok) memcpy(q->ttok + q->ttok0, o->tgt_tok, sizeof(int32_t) * (size_t)o->n_tgt_tok);
  if (o->n_truth) {
    memcpy(q->trs + q->truth0, o->truth_src, sizeof(int32_t) * (size_t)o->n_truth);
    memcpy(q->trt + q->truth0, o->truth_tgt, sizeof(int32_t) * (size_t)o->n_truth);
  }
  return NULL;
}

/* Copy a job's parts into the caller's arrays (sizes from the totals;
 * offsets arrays hold n+1 entries) and release the job. */
int synth_collect(void *job, int64_t *src_doc_off, int64_t *src_sent_off, int32_t *src_tok, int64_t *tgt_doc_off,
                  int64_t *tgt_sent_off, int32_t *tgt_tok, int64_t *truth_off, int32_t *truth_src,
                  int32_t *truth_tgt) {
  synth_job *j = (synth_job *)job;
  if (!j) return -1;
  const int T = j->n_parts;
  collect_part *cp = (collect_part *)calloc((size_t)T, sizeof(collect_part));
  pthread_t *th = (pthread_t *)calloc((size_t)T, sizeof(pthread_t));
  if (!cp || !th) {
    free(cp);
    free(th);
    job_free(j);
    return -1;
  }
  src_doc_off[0] = tgt_doc_off[0] = truth_off[0] = 0;
  src_sent_off[0] = tgt_sent_off[0] = 0;
  int64_t b[6] = {0, 0, 0, 0, 0, 0};
  for (int k = 0; k < T; k++) {
    const synth_corpus *o = &j->parts[k].out;
    collect_part x = {o, b[0], b[1], b[2], b[3], b[4], b[5], src_doc_off, src_sent_off, tgt_doc_off, tgt_sent_off,
                      truth_off, src_tok, tgt_tok, truth_src, truth_tgt};
    cp[k] = x;
    b[0] += o->n_pairs;
    b[1] += o->n_src_sent;
    b[2] += o->n_tgt_sent;
    b[3] += o->n_src_tok;
    b[4] += o->n_tgt_tok;
    b[5] += o->n_truth;
  }
  for (int k = 1; k < T; k++)
    if (pthread_create(&th[k], NULL, collect_run, &cp[k]) != 0) {
      collect_run(&cp[k]);
      th[k] = 0;
    }
  collect_run(&cp[0]);
  for (int k = 1; k < T; k++)
    if (th[k]) pthread_join(th[k], NULL);
  free(cp);
  free(th);
  job_free(j);
  return 0;
}

/*
 * Bilingual lexicon as CSR over entries (src id, list of target ids).
 * Source ids: `n_translated` ids chosen uniformly from [0, V) (all of them when
 * n_translated >= V).  Each gets k ~ U{kmin..kmax} distinct targets; the first
 * is the id itself (frequent words translate to frequent words), the rest are
 * uniform.  When the translation pairs fall short of `n_pairs_total`, decoy
 * keys V, V+1, ... (ids that never occur in text) are added until the table
 * holds that many pairs.  Output arrays are malloc'ed; release with free via
 * synth_free_lexicon.
 */
typedef struct {
  int64_t n_src;
  int32_t *src_ids;
  int64_t *off;
  int32_t *tgt_ids;
  int64_t n_tgt;
} synth_lexicon;

int synth_free_lexicon(synth_lexicon *L) {
  free(L->src_ids);
  free(L->off);
  free(L->tgt_ids);
  memset(L, 0, sizeof(*L));
  return 0;
}

int synth_make_lexicon(int32_t V, int64_t n_translated, int32_t kmin, int32_t kmax, int64_t n_pairs_total,
                       uint64_t seed, synth_lexicon *L) {
  memset(L, 0, sizeof(*L));
  if (V <= 0 || kmin < 1 || kmax < kmin) return -2;
  if (n_translated > V) n_translated = V;
  rng_t r = rng_make(seed, 0xfffffff1ULL, 11);
  /* choose translated ids: partial Fisher-Yates over [0, V) */
  int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)V);
  if (!ids) return -1;
  for (int32_t i = 0; i < V; i++) ids[i] = i;
  for (int64_t k = 0; k < n_translated; k++) {
    int64_t j = rng_int(&r, k, V - 1);
    int32_t t = ids[k];
    ids[k] = ids[j];
    ids[j] = t;
  }
  /* mark and emit in id order */
  char *mark = (char *)calloc((size_t)V, 1);
  if (!mark) {
    free(ids);
    return -1;
  }
  for (int64_t k = 0; k < n_translated; k++) mark[ids[k]] = 1;
  free(ids);

  vec32 src = {0}, tgt = {0};
  vec64 off = {0};
  int rc = v64_push(&off, 0);
  int32_t sel[64];
  for (int32_t x = 0; x < V && !rc; x++) {
    if (!mark[x]) continue;
    int32_t k = (int32_t)rng_int(&r, kmin, kmax);
    if (k > 64) k = 64;
    sel[0] = x;
    int32_t have = 1;
    while (have < k) {
      int32_t y = (int32_t)rng_int(&r, 0, V - 1);
      int dup = 0;
      for (int32_t e = 0; e < have; e++) dup |= (sel[e] == y);
      if (!dup) sel[have++] = y;
    }
    rc |= v32_push(&src, x);
    for (int32_t e = 0; e < k; e++) rc |= v32_push(&tgt, sel[e]);
    rc |= v64_push(&off, tgt.n);
  }
  free(mark);
  /* decoys */
  int64_t decoy = V;
  while (!rc && tgt.n < n_pairs_total && decoy < 0x7fffffffLL) {
    int32_t k = (int32_t)rng_int(&r, kmin, kmax);
    if (k > 64) k = 64;
    if (tgt.n + k > n_pairs_total) k = (int32_t)(n_pairs_total - tgt.n);
    int32_t have = 0;
    while (have < k) {
      int32_t y = (int32_t)rng_int(&r, 0, V - 1);
      int dup = 0;
      for (int32_t e = 0; e < have; e++) dup |= (sel[e] == y);
      if (!dup) sel[have++] = y;
    }
    rc |= v32_push(&src, (int32_t)decoy++);
    for (int32_t e = 0; e < k; e++) rc |= v32_push(&tgt, sel[e]);
    rc |= v64_push(&off, tgt.n);
  }
  if (rc) {
    free(src.p);
    free(tgt.p);
    free(off.p);
    return -1;
  }
  L->n_src = src.n;
  L->src_ids = src.p;
  L->off = off.p;
  L->tgt_ids = tgt.p;
  L->n_tgt = tgt.n;
  return 0;
}

/* Classifier weights: w0 ~ U[-7,-5], w1, w2 ~ U[4.5,6.5], w3 ~ U[0.5,1.5]. */
void synth_weights(uint64_t seed, float w[4]) {
  rng_t r = rng_make(seed, 0xfffffff2ULL, 12);
  w[0] = (float)(-7.0 + 2.0 * rng_unif(&r));
  w[1] = (float)(4.5 + 2.0 * rng_unif(&r));
  w[2] = (float)(4.5 + 2.0 * rng_unif(&r));
  w[3] = (float)(0.5 + 1.0 * rng_unif(&r));
}

/* Poisson arrivals: n times (seconds) with rate `rate` per second. */
void synth_arrivals(uint64_t seed, double rate, int64_t n, double *t) {
  rng_t r = rng_make(seed, 0xfffffff3ULL, 13);
  double acc = 0.0;
  for (int64_t k = 0; k < n; k++) {
    double u = rng_unif(&r);
    if (u < 0x1.0p-60) u = 0x1.0p-60;
    acc += -log(u) / rate;
    t[k] = acc;
  }
}

/* Uniform draws for the tests' random small cases: n ints in [lo, hi]. */
void synth_uniform_ints(uint64_t seed, uint64_t stream, int64_t n, int64_t lo, int64_t hi, int64_t *out) {
  rng_t r = rng_make(seed, stream, 14);
  for (int64_t k = 0; k < n; k++) out[k] = rng_int(&r, lo, hi);
}
