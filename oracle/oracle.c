/*
 * CPU oracle for the comparable-corpus miner (test infrastructure only).
 *
 * This file is the plain, slow, single-threaded statement of what the miner
 * computes.  It exists to check the GPU library; the product never calls it.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load it.  It shares no code, header or table with the GPU library.
 *
 * Build: gcc -O2 -std=gnu99 -ffp-contract=off -fno-fast-math -pthread (no FMA
 * contraction: every float product and sum below is rounded on its own).  The
 * per-pair functions are single-threaded; oracle_mine_threads at the end only
 * hands whole pairs to worker threads.
 *
 * The method (Section 4, "Yalign and improvements"):
 *   - every source sentence of a document pair is scored against every target
 *     sentence by a classifier whose confidence is a probability; these scores
 *     form the matrix that the aligner walks;
 *   - the matrix is aligned with Needleman-Wunsch instead of A* search; the
 *     path may not move up or left, and a penalty controls skipping ahead;
 *   - a matched sentence pair is accepted when its confidence reaches the
 *     threshold.
 * The classifier is a fixed linear model over lexicon-overlap and length
 * features followed by the logistic function (a Platt-scaled SVM decision
 * value has that form).  Readings of points the paper leaves open are marked
 * [reading] below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------- lexicon */
/*
 * Bilingual lexicon T: source id -> set of target ids.  Stored as the sorted,
 * duplicate-free list of (source id, target id) pairs; an id that is absent
 * has the empty set.  Entries listing the same source id twice are merged
 * [reading: duplicates and order carry no meaning].
 */
typedef struct {
  int64_t n;
  int32_t *key;
  int32_t *tgt;
} olex;

static int cmp_pair(const void *a, const void *b) {
  const int32_t *x = (const int32_t *)a, *y = (const int32_t *)b;
  if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
  if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1;
  return 0;
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

int oracle_lex_build(const int32_t *src_ids, const int64_t *off, const int32_t *tgt_ids, int64_t n_src,
                     olex **out) {
  *out = NULL;
  int64_t total = n_src > 0 ? off[n_src] - off[0] : 0;
  int32_t *pairs = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)(total > 0 ? total : 1));
  if (!pairs) return -1;
  int64_t k = 0;
  for (int64_t e = 0; e < n_src; e++)
    for (int64_t v = off[e]; v < off[e + 1]; v++) {
      pairs[2 * k] = src_ids[e];
      pairs[2 * k + 1] = tgt_ids[v];
      k++;
    }
  qsort(pairs, (size_t)k, 2 * sizeof(int32_t), cmp_pair);
  olex *L = (olex *)calloc(1, sizeof(olex));
  L->key = (int32_t *)malloc(sizeof(int32_t) * (size_t)(k > 0 ? k : 1));
  L->tgt = (int32_t *)malloc(sizeof(int32_t) * (size_t)(k > 0 ? k : 1));
  int64_t u = 0;
  for (int64_t e = 0; e < k; e++) {
    if (u > 0 && L->key[u - 1] == pairs[2 * e] && L->tgt[u - 1] == pairs[2 * e + 1]) continue;
    L->key[u] = pairs[2 * e];
    L->tgt[u] = pairs[2 * e + 1];
    u++;
  }
  L->n = u;
  free(pairs);
  *out = L;
  return 0;
}

void oracle_lex_free(olex *L) {
  if (!L) return;
  free(L->key);
  free(L->tgt);
  free(L);
}

/* T(x) as the index range [*lo, *hi) of the sorted pair list. */
static void lex_range(const olex *L, int32_t x, int64_t *lo, int64_t *hi) {
  int64_t a = 0, b = L->n;
  while (a < b) {
    int64_t mid = a + (b - a) / 2;
    if (L->key[mid] < x)
      a = mid + 1;
    else
      b = mid;
  }
  *lo = a;
  b = L->n;
  while (a < b) {
    int64_t mid = a + (b - a) / 2;
    if (L->key[mid] <= x)
      a = mid + 1;
    else
      b = mid;
  }
  *hi = a;
}

static int in_sorted(const int32_t *set, int64_t n, int32_t x) {
  return n > 0 && bsearch(&x, set, (size_t)n, sizeof(int32_t), cmp_i32) != NULL;
}

/* sorted, duplicate-free copy of a[0..n); returns its length */
static int64_t sorted_unique(int32_t *dst, const int32_t *a, int64_t n) {
  memcpy(dst, a, sizeof(int32_t) * (size_t)n);
  qsort(dst, (size_t)n, sizeof(int32_t), cmp_i32);
  int64_t u = 0;
  for (int64_t k = 0; k < n; k++)
    if (u == 0 || dst[u - 1] != dst[k]) dst[u++] = dst[k];
  return u;
}

/* ---------------------------------------------------------- similarity */
/*
 * Sentence-pair score matrix of one document pair (the matrix the aligner
 * walks, Section 4).  Source sentence i has a_i tokens, target sentence j has
 * b_j tokens.
 *
 *   X_i     = union over the tokens x of sentence i of T(x)   (set of target ids)
 *   m_t(i,j) = number of target positions p with t_j[p] in X_i
 *   m_s(i,j) = number of source positions q with T(s_i[q]) meeting the token
 *              set of t_j
 *   [reading: positions are counted with multiplicity, ids as sets]
 *   f1 = m_s / a_i,  f2 = m_t / b_j,  f3 = min(a_i, b_j) / max(a_i, b_j)
 *        (float division; a zero denominator gives 0)
 *   z  = ((w0 + w1*f1) + w2*f2) + w3*f3     (float, left to right, no FMA)
 *   S  = 1 / (1 + exp(-z))                  (in double, rounded once to float)
 *
 * S is row-major n x m.  m_s and m_t (n x m) are optional.
 * src_sent_off has n+1 absolute offsets into src_tok; same for the target.
 */
static float ratio(int32_t num, int32_t den) { return den == 0 ? 0.0f : (float)num / (float)den; }

float oracle_score(const float w[4], int32_t ms, int32_t a, int32_t mt, int32_t b) {
  float f1 = ratio(ms, a);
  float f2 = ratio(mt, b);
  int32_t lo = a < b ? a : b, hi = a < b ? b : a;
  float f3 = ratio(lo, hi);
  float z = w[0];
  float t = w[1] * f1;
  z = z + t;
  t = w[2] * f2;
  z = z + t;
  t = w[3] * f3;
  z = z + t;
  return (float)(1.0 / (1.0 + exp(-(double)z)));
}

int oracle_similarity(const olex *L, const int64_t *src_sent_off, const int32_t *src_tok, int32_t n,
                      const int64_t *tgt_sent_off, const int32_t *tgt_tok, int32_t m, const float w[4],
                      float *S, int32_t *m_s_out, int32_t *m_t_out) {
  if (n <= 0 || m <= 0) return 0;
  /* X_i for every source sentence, and the token set of every target sentence */
  int32_t **X = (int32_t **)calloc((size_t)n, sizeof(int32_t *));
  int64_t *nX = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  int32_t **Y = (int32_t **)calloc((size_t)m, sizeof(int32_t *));
  int64_t *nY = (int64_t *)calloc((size_t)m, sizeof(int64_t));
  if (!X || !nX || !Y || !nY) return -1;
  for (int32_t i = 0; i < n; i++) {
    int64_t tot = 0;
    for (int64_t q = src_sent_off[i]; q < src_sent_off[i + 1]; q++) {
      int64_t lo, hi;
      lex_range(L, src_tok[q], &lo, &hi);
      tot += hi - lo;
    }
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tot + 1));
    int64_t k = 0;
    for (int64_t q = src_sent_off[i]; q < src_sent_off[i + 1]; q++) {
      int64_t lo, hi;
      lex_range(L, src_tok[q], &lo, &hi);
      for (int64_t e = lo; e < hi; e++) buf[k++] = L->tgt[e];
    }
    X[i] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tot + 1));
    nX[i] = sorted_unique(X[i], buf, k);
    free(buf);
  }
  for (int32_t j = 0; j < m; j++) {
    int64_t b = tgt_sent_off[j + 1] - tgt_sent_off[j];
    Y[j] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(b + 1));
    nY[j] = sorted_unique(Y[j], tgt_tok + tgt_sent_off[j], b);
  }
  for (int32_t i = 0; i < n; i++) {
    int32_t a = (int32_t)(src_sent_off[i + 1] - src_sent_off[i]);
    for (int32_t j = 0; j < m; j++) {
      int32_t b = (int32_t)(tgt_sent_off[j + 1] - tgt_sent_off[j]);
      int32_t mt = 0, ms = 0;
      for (int64_t p = tgt_sent_off[j]; p < tgt_sent_off[j + 1]; p++)
        if (in_sorted(X[i], nX[i], tgt_tok[p])) mt++;
      for (int64_t q = src_sent_off[i]; q < src_sent_off[i + 1]; q++) {
        int64_t lo, hi;
        lex_range(L, src_tok[q], &lo, &hi);
        for (int64_t e = lo; e < hi; e++)
          if (in_sorted(Y[j], nY[j], L->tgt[e])) {
            ms++;
            break;
          }
      }
      S[(int64_t)i * m + j] = oracle_score(w, ms, a, mt, b);
      if (m_s_out) m_s_out[(int64_t)i * m + j] = ms;
      if (m_t_out) m_t_out[(int64_t)i * m + j] = mt;
    }
  }
  for (int32_t i = 0; i < n; i++) free(X[i]);
  for (int32_t j = 0; j < m; j++) free(Y[j]);
  free(X);
  free(nX);
  free(Y);
  free(nY);
  return 0;
}

/* ------------------------------------------------------ Needleman-Wunsch */
/*
 * Global alignment of the source and target sentence sequences over S
 * (Section 4: Needleman-Wunsch replaces A*; the path never goes up or left;
 * the penalty controls skipping ahead).  In float:
 *   H[0][0] = 0
 *   H[i][0] = H[i-1][0] + g   (move U; repeated addition, not i*g)
 *   H[0][j] = H[0][j-1] + g   (move L)
 *   H[i][j] = best of  D: H[i-1][j-1] + S[i-1][j-1]
 *                      U: H[i-1][j]   + g   (source sentence i-1 unaligned)
 *                      L: H[i][j-1]   + g   (target sentence j-1 unaligned)
 * taking D first and switching only on a strictly greater value, U before L
 * [reading: a fixed tie rule D > U > L].
 * The traceback walks back from (n, m) to (0, 0); `moves` receives the path in
 * forward order (n_moves = #D + #U + #L).  H ((n+1) x (m+1), optional)
 * receives the full matrix.
 */
int oracle_nw(const float *S, int32_t n, int32_t m, float g, float *H_out, char *moves, int32_t *n_moves,
              float *h_nm) {
  int64_t W = (int64_t)m + 1;
  float *H = (float *)malloc(sizeof(float) * (size_t)((int64_t)(n + 1) * W));
  char *dir = (char *)malloc((size_t)((int64_t)(n + 1) * W));
  if (!H || !dir) {
    free(H);
    free(dir);
    return -1;
  }
  H[0] = 0.0f;
  dir[0] = 0;
  for (int32_t i = 1; i <= n; i++) {
    H[i * W] = H[(i - 1) * W] + g;
    dir[i * W] = 'U';
  }
  for (int32_t j = 1; j <= m; j++) {
    H[j] = H[j - 1] + g;
    dir[j] = 'L';
  }
  for (int32_t i = 1; i <= n; i++)
    for (int32_t j = 1; j <= m; j++) {
      float d = H[(i - 1) * W + (j - 1)] + S[(int64_t)(i - 1) * m + (j - 1)];
      float u = H[(i - 1) * W + j] + g;
      float l = H[i * W + (j - 1)] + g;
      float best = d;
      char c = 'D';
      if (u > best) {
        best = u;
        c = 'U';
      }
      if (l > best) {
        best = l;
        c = 'L';
      }
      H[i * W + j] = best;
      dir[i * W + j] = c;
    }
  if (h_nm) *h_nm = H[(int64_t)n * W + m];
  if (H_out) memcpy(H_out, H, sizeof(float) * (size_t)((int64_t)(n + 1) * W));
  /* traceback */
  int32_t i = n, j = m, k = 0;
  char *rev = (char *)malloc((size_t)(n + m + 1));
  while (i > 0 || j > 0) {
    char c = dir[(int64_t)i * W + j];
    rev[k++] = c;
    if (c == 'D') {
      i--;
      j--;
    } else if (c == 'U') {
      i--;
    } else {
      j--;
    }
  }
  for (int32_t e = 0; e < k; e++) moves[e] = rev[k - 1 - e];
  *n_moves = k;
  free(rev);
  free(H);
  free(dir);
  return 0;
}

/*
 * Threshold filter (Section 4: an alignment is accepted as good when its
 * confidence reaches the threshold).  Every D move into cell (i+1, j+1) of the
 * path pairs source sentence i with target sentence j; it is kept when
 * S[i][j] >= tau [reading: equality accepted; only matched cells of the path
 * are candidates].  Pairs come out in path order.
 */
int oracle_emit(const float *S, int32_t n, int32_t m, const char *moves, int32_t n_moves, float tau,
                int32_t *src_idx, int32_t *tgt_idx, float *score, int32_t *count) {
  (void)n;
  int32_t i = 0, j = 0, c = 0;
  for (int32_t k = 0; k < n_moves; k++) {
    if (moves[k] == 'D') {
      float s = S[(int64_t)i * m + j];
      if (s >= tau) {
        src_idx[c] = i;
        tgt_idx[c] = j;
        score[c] = s;
        c++;
      }
      i++;
      j++;
    } else if (moves[k] == 'U') {
      i++;
    } else {
      j++;
    }
  }
  *count = c;
  return 0;
}

/*
 * The whole miner over a packed batch of document pairs (three-level CSR:
 * pair -> sentences -> tokens, int64 offsets).  Results are written compactly:
 * pair p's accepted pairs occupy [pair_off[p], pair_off[p+1]) of src_idx,
 * tgt_idx, score (capacity: sum over pairs of min(n, m)); align_score[p] is
 * H[n][m].  S_out (optional) receives every pair's score matrix back to back.
 */
int oracle_mine(const olex *L, int64_t n_pairs, const int64_t *src_doc_off, const int64_t *src_sent_off,
                const int32_t *src_tok, const int64_t *tgt_doc_off, const int64_t *tgt_sent_off,
                const int32_t *tgt_tok, const float w[4], float g, float tau, int64_t *pair_off,
                int32_t *src_idx, int32_t *tgt_idx, float *score, float *align_score, float *S_out) {
  int64_t out = 0, s_base = 0;
  pair_off[0] = 0;
  for (int64_t p = 0; p < n_pairs; p++) {
    int32_t n = (int32_t)(src_doc_off[p + 1] - src_doc_off[p]);
    int32_t m = (int32_t)(tgt_doc_off[p + 1] - tgt_doc_off[p]);
    int64_t cells = (int64_t)n * m;
    float *S = (float *)malloc(sizeof(float) * (size_t)(cells > 0 ? cells : 1));
    char *mv = (char *)malloc((size_t)(n + m + 1));
    if (!S || !mv) return -1;
    if (oracle_similarity(L, src_sent_off + src_doc_off[p], src_tok, n, tgt_sent_off + tgt_doc_off[p], tgt_tok,
                          m, w, S, NULL, NULL))
      return -1;
    int32_t nm = 0, c = 0;
    float h = 0.0f;
    if (oracle_nw(S, n, m, g, NULL, mv, &nm, &h)) return -1;
    oracle_emit(S, n, m, mv, nm, tau, src_idx + out, tgt_idx + out, score + out, &c);
    out += c;
    pair_off[p + 1] = out;
    align_score[p] = h;
    if (S_out) memcpy(S_out + s_base, S, sizeof(float) * (size_t)cells);
    s_base += cells;
    free(S);
    free(mv);
  }
  return 0;
}

/*
 * Multi-threaded driver: the same per-pair computation as oracle_mine, with
 * pairs handed to worker threads one at a time (the multi-threaded Yalign of
 * Section 4 parallelises over article pairs the same way).  Each pair's
 * accepted pairs go to its own slot range (prefix sums of min(n, m)); the
 * caller-visible output is compacted afterwards exactly as oracle_mine's.
 */
#include <pthread.h>

typedef struct {
  const olex *L;
  int64_t n_pairs;
  const int64_t *sdo, *sso, *tdo, *tso;
  const int32_t *stok, *ttok;
  const float *w;
  float g, tau;
  const int64_t *slot_off;
  int32_t *ssrc, *stgt;
  float *sscore, *align;
  int32_t *cnt;
  volatile int64_t next;
  volatile int failed;
} mt_job;

static void *mt_worker(void *arg) {
  mt_job *J = (mt_job *)arg;
  for (;;) {
    const int64_t p = __sync_fetch_and_add(&J->next, 1);
    if (p >= J->n_pairs) break;
    const int32_t n = (int32_t)(J->sdo[p + 1] - J->sdo[p]), m = (int32_t)(J->tdo[p + 1] - J->tdo[p]);
    const int64_t cells = (int64_t)n * m;
    float *S = (float *)malloc(sizeof(float) * (size_t)(cells > 0 ? cells : 1));
    char *mv = (char *)malloc((size_t)(n + m + 1));
    int32_t nm = 0, c = 0;
    float h = 0.0f;
    if (!S || !mv || oracle_similarity(J->L, J->sso + J->sdo[p], J->stok, n, J->tso + J->tdo[p], J->ttok, m, J->w, S, NULL, NULL) ||
        oracle_nw(S, n, m, J->g, NULL, mv, &nm, &h)) {
      J->failed = 1;
    } else {
      const int64_t o = J->slot_off[p];
      oracle_emit(S, n, m, mv, nm, J->tau, J->ssrc + o, J->stgt + o, J->sscore + o, &c);
      J->cnt[p] = c;
      J->align[p] = h;
    }
    free(S);
    free(mv);
  }
  return NULL;
}

int oracle_mine_threads(const olex *L, int64_t n_pairs, const int64_t *src_doc_off, const int64_t *src_sent_off,
                        const int32_t *src_tok, const int64_t *tgt_doc_off, const int64_t *tgt_sent_off,
                        const int32_t *tgt_tok, const float w[4], float g, float tau, int n_threads, int64_t *pair_off,
                        int32_t *src_idx, int32_t *tgt_idx, float *score, float *align_score) {
  if (n_threads < 1) n_threads = 1;
  int64_t *slot_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_pairs + 1));
  int32_t *cnt = (int32_t *)calloc((size_t)(n_pairs > 0 ? n_pairs : 1), sizeof(int32_t));
  if (!slot_off || !cnt) return -1;
  slot_off[0] = 0;
  for (int64_t p = 0; p < n_pairs; p++) {
    const int64_t n = src_doc_off[p + 1] - src_doc_off[p], m = tgt_doc_off[p + 1] - tgt_doc_off[p];
    slot_off[p + 1] = slot_off[p] + (n < m ? n : m);
  }
  const int64_t cap = slot_off[n_pairs] > 0 ? slot_off[n_pairs] : 1;
  int32_t *ssrc = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
  int32_t *stgt = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
  float *sscore = (float *)malloc(sizeof(float) * (size_t)cap);
  if (!ssrc || !stgt || !sscore) return -1;
  mt_job J = {L, n_pairs, src_doc_off, src_sent_off, tgt_doc_off, tgt_sent_off, src_tok, tgt_tok, w, g, tau,
              slot_off, ssrc, stgt, sscore, align_score, cnt, 0, 0};
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
  for (int t = 0; t < n_threads; t++) pthread_create(&th[t], NULL, mt_worker, &J);
  for (int t = 0; t < n_threads; t++) pthread_join(th[t], NULL);
  free(th);
  int64_t out = 0;
  pair_off[0] = 0;
  for (int64_t p = 0; p < n_pairs; p++) {
    for (int32_t k = 0; k < cnt[p]; k++) {
      src_idx[out] = ssrc[slot_off[p] + k];
      tgt_idx[out] = stgt[slot_off[p] + k];
      score[out] = sscore[slot_off[p] + k];
      out++;
    }
    pair_off[p + 1] = out;
  }
  const int failed = J.failed;
  free(slot_off);
  free(cnt);
  free(ssrc);
  free(stgt);
  free(sscore);
  return failed ? -1 : 0;
}
