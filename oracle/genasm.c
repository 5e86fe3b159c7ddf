/*
 * GenASM (bitap with traceback), windowed.  TEST INFRASTRUCTURE ONLY: the
 * plain CPU form of the GenASM alignment the GPU library computes.  It
 * shares no code with the other oracle files nor with the GPU library.
 *
 * Paper: System and Methods, "GenASM": the bitap algorithm extended with a
 * traceback; the input includes the largest number of edits k the alignment
 * may use; each thread keeps a bit-mask of the pattern per alphabet
 * character, two status bit-vectors (the previous and the current text
 * position) and four intermediate bit-vectors, one per edit case (match,
 * substitution, deletion, insertion).  The rest is not in the paper (the
 * cited GenASM work defines it); the reading this file writes out:
 *
 * Edits.  Unit costs: '=' 0, 'X', 'I' (a pattern base alone), 'D' (a text
 * base alone) 1 each.  The score is the number of edits of the alignment
 * produced; the threshold is k (< 0: none).
 *
 * Windows.  The pair is aligned from its end towards its start in windows
 * of at most W pattern and W text bases.  With (me, ne) the bases still to
 * align (initially (m, n)), a window takes the last a = min(W, me) pattern
 * and b = min(W, ne) text bases of that prefix.  It is the final window when
 * me <= W and ne <= W: then its alignment must start at the start of both
 * sequences (anchored); otherwise it may start anywhere on its first row or
 * column (free), the part before it being left to later windows.
 *
 * Distance calculation (bitap) in a window, pattern p_1..p_a, text
 * t_1..t_b: with D(i, j) the fewest edits aligning p_1..p_i with t_1..t_j
 * (start cells D(i, 0) = i and D(0, j) = j when anchored, 0 when free), the
 * status bit-vector of text position j at edit level d holds bit i =
 * [D(i, j) <= d].  Bit 0 is the start row and is known without computation.
 * For j = 1..b and, within it, d = 0..Lw, from the status of j - 1 ("old")
 * and of j ("new", lower levels):
 *   match        = PM[t_j]_i and old_d[i-1]
 *   substitution = old_{d-1}[i-1]
 *   insertion    = new_{d-1}[i-1]    (p_i alone)
 *   deletion     = old_{d-1}[i]      (t_j alone)
 *   new_d[i]     = match | substitution | insertion | deletion
 * (the d - 1 terms are absent at level 0).  The window's distance is the
 * least d with bit a set at j = b.  Lw = max(a, b), capped at k minus the
 * edits already committed when k >= 0; no level up to Lw reaching bit a
 * rejects the pair.
 *
 * Traceback, from (a, b) backwards with a budget of d edits (initially the
 * window's distance), using the intermediate vectors stored by the
 * distance calculation at (j, d): the first available of
 *   1. 'I' if the previous op (the one to its right) was 'I' and insertion
 *      is set; 2. 'D' likewise for deletion -- a gap run is extended before
 *      anything else (the affine flavour of the traceback);
 *   3. '=' if match is set; 4. 'X' if substitution is set (then p_i != t_j,
 *      else 3 applied); 5. 'I'; 6. 'D'.
 * Edits lower the budget by one.  On the start row (i = 0) only 'D' is
 * available and on the start column (j = 0) only 'I'.  The walk commits ops
 * until it reaches the window's start (final window) or, for other windows,
 * until it has consumed at least C = W - O bases of either sequence or
 * reached the window's first row or column; the committed ops' bases leave
 * (me, ne).  When me or ne reaches 0 the other's remaining bases become 'I'
 * (or 'D') ops.  The pair is rejected when its edits exceed k.
 *
 * Rejected pairs: score -1, no runs.  Runs are `len << 4 | op`, first op
 * first (ops '=' 0, 'X' 1, 'I' 2, 'D' 3).
 *
 * Work counters (the units in which the GPU kernel's work is stated), when
 * `stats` is not NULL: stats[0] windows aligned, stats[1] status-vector
 * updates the distance calculation needs -- (distance + 1) x b per window,
 * the levels up to the one that reaches bit a at every text position --
 * stats[2] traceback steps (ops committed inside windows).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { G_EQ = 0, G_X = 1, G_I = 2, G_D = 3, G_NONE = 4 };

/* Status bits [D(i, j) <= d] of one window for j = 0..b, d = 0..L,
 * i = 0..a, one byte per bit, and the four intermediate vectors of each
 * (j >= 1, d). */
typedef struct {
  int32_t a, b, L;
  uint8_t *R, *Mt, *Sb, *In, *De;
} window_dc;

static size_t at(const window_dc *w, int32_t j, int32_t d, int32_t i) {
  return ((size_t)j * (size_t)(w->L + 1) + (size_t)d) * (size_t)(w->a + 1) + (size_t)i;
}

/* Start-row bit: [D(0, j) <= d]. */
static uint8_t start_row(int anchored, int32_t j, int32_t d) { return anchored ? (uint8_t)(j <= d) : 1; }

/* Distance calculation of one window (levels 0..L).  Returns 0, or -1 when
 * out of memory. */
static int dc_window(window_dc *w, const uint8_t *p, int32_t a, const uint8_t *t, int32_t b, int anchored,
                     int32_t L) {
  w->a = a;
  w->b = b;
  w->L = L;
  const size_t cells = (size_t)(b + 1) * (size_t)(L + 1) * (size_t)(a + 1);
  w->R = (uint8_t *)calloc(cells, 1);
  w->Mt = (uint8_t *)calloc(cells, 1);
  w->Sb = (uint8_t *)calloc(cells, 1);
  w->In = (uint8_t *)calloc(cells, 1);
  w->De = (uint8_t *)calloc(cells, 1);
  if (!w->R || !w->Mt || !w->Sb || !w->In || !w->De) return -1;
  /* pattern bit-masks: PM[c][i] = [p_i == c] */
  uint8_t *PM = (uint8_t *)calloc((size_t)4 * (size_t)(a + 1), 1);
  if (!PM) return -1;
  for (int32_t i = 1; i <= a; ++i) PM[(size_t)p[i - 1] * (size_t)(a + 1) + (size_t)i] = 1;
  /* status before any text: [D(i, 0) <= d] */
  for (int32_t d = 0; d <= L; ++d)
    for (int32_t i = 0; i <= a; ++i) w->R[at(w, 0, d, i)] = anchored ? (uint8_t)(i <= d) : 1;
  for (int32_t j = 1; j <= b; ++j) {
    const uint8_t *pm = PM + (size_t)t[j - 1] * (size_t)(a + 1);
    for (int32_t d = 0; d <= L; ++d) {
      w->R[at(w, j, d, 0)] = start_row(anchored, j, d);
      for (int32_t i = 1; i <= a; ++i) {
        const uint8_t mt = pm[i] & w->R[at(w, j - 1, d, i - 1)];
        uint8_t sb = 0, in = 0, de = 0;
        if (d > 0) {
          sb = w->R[at(w, j - 1, d - 1, i - 1)];
          in = w->R[at(w, j, d - 1, i - 1)];
          de = w->R[at(w, j - 1, d - 1, i)];
        }
        w->Mt[at(w, j, d, i)] = mt;
        w->Sb[at(w, j, d, i)] = sb;
        w->In[at(w, j, d, i)] = in;
        w->De[at(w, j, d, i)] = de;
        w->R[at(w, j, d, i)] = (uint8_t)(mt | sb | in | de);
      }
    }
  }
  free(PM);
  return 0;
}

static void dc_free(window_dc *w) {
  free(w->R);
  free(w->Mt);
  free(w->Sb);
  free(w->In);
  free(w->De);
  memset(w, 0, sizeof(*w));
}

/* Status bits of one window for the tests: out[(j * (L + 1) + d) * (a + 1)
 * + i] = [D(i, j) <= d]. */
int oracle_genasm_dc(const uint8_t *p, int32_t a, const uint8_t *t, int32_t b, int32_t anchored, int32_t L,
                     uint8_t *out) {
  window_dc w;
  memset(&w, 0, sizeof(w));
  if (a < 0 || b < 0 || L < 0) return -2;
  if (dc_window(&w, p, a, t, b, anchored != 0, L)) {
    dc_free(&w);
    return -1;
  }
  memcpy(out, w.R, (size_t)(b + 1) * (size_t)(L + 1) * (size_t)(a + 1));
  dc_free(&w);
  return 0;
}

int oracle_genasm(const uint8_t *P, int32_t m, const uint8_t *T, int32_t n, int32_t k, int32_t W, int32_t Ov,
                  int32_t want_cigar, int32_t *score, int8_t *status, uint32_t *runs, int32_t cap,
                  int32_t *nruns, int64_t *stats) {
  if (m < 0 || n < 0 || W < 1 || Ov < 0 || Ov >= W) return -2;
  if (stats) stats[0] = stats[1] = stats[2] = 0;
  const int32_t C = W - Ov;
  /* ops, last op first */
  uint8_t *rev = (uint8_t *)malloc((size_t)m + (size_t)n + 1);
  if (!rev) return -1;
  int32_t nops = 0, used = 0, me = m, ne = n, prev = G_NONE, rejected = 0;
  while (me > 0 && ne > 0 && !rejected) {
    const int anchored = me <= W && ne <= W;
    const int32_t a = me < W ? me : W, b = ne < W ? ne : W;
    int32_t L = a > b ? a : b;
    if (k >= 0 && k - used < L) L = k - used;
    window_dc w;
    memset(&w, 0, sizeof(w));
    if (dc_window(&w, P + (me - a), a, T + (ne - b), b, anchored, L)) {
      dc_free(&w);
      free(rev);
      return -1;
    }
    int32_t d = 0;
    while (d <= L && !w.R[at(&w, b, d, a)]) ++d;
    if (d > L) {
      rejected = 1;
      dc_free(&w);
      break;
    }
    if (stats) {
      stats[0] += 1;
      stats[1] += (int64_t)(d + 1) * b;
    }
    int32_t i = a, j = b;
    for (;;) {
      if (anchored) {
        if (i == 0 && j == 0) break;
      } else if (a - i >= C || b - j >= C || i == 0 || j == 0) {
        break;
      }
      int op;
      if (i == 0) {
        op = G_D;
      } else if (j == 0) {
        op = G_I;
      } else {
        const size_t c = at(&w, j, d, i);
        if (prev == G_I && w.In[c]) op = G_I;
        else if (prev == G_D && w.De[c]) op = G_D;
        else if (w.Mt[c]) op = G_EQ;
        else if (w.Sb[c]) op = G_X;
        else if (w.In[c]) op = G_I;
        else op = G_D; /* deletion: the status bit is set, so one case is */
      }
      if (op != G_EQ) d -= 1, used += 1;
      if (op != G_D) i -= 1;
      if (op != G_I) j -= 1;
      rev[nops++] = (uint8_t)op;
      prev = op;
      if (stats) stats[2] += 1;
    }
    me -= a - i;
    ne -= b - j;
    dc_free(&w);
  }
  if (!rejected) {
    for (; me > 0; --me) rev[nops++] = G_I, ++used;
    for (; ne > 0; --ne) rev[nops++] = G_D, ++used;
    if (k >= 0 && used > k) rejected = 1;
  }
  *nruns = 0;
  if (rejected) {
    *score = -1;
    *status = 1;
    free(rev);
    return 0;
  }
  *score = used;
  *status = 0;
  if (want_cigar) {
    int32_t nr = 0;
    for (int32_t q = nops - 1; q >= 0;) {
      int32_t r = q;
      while (r >= 0 && rev[r] == rev[q]) --r;
      if (nr >= cap) {
        free(rev);
        return -3;
      }
      runs[nr++] = ((uint32_t)(q - r) << 4) | rev[q];
      q = r;
    }
    *nruns = nr;
  }
  free(rev);
  return 0;
}

/* Batch driver: pairs are independent; a pthread pool takes chunks of
 * consecutive pairs. */
typedef struct {
  int64_t n;
  const uint8_t *pat, *txt;
  const int64_t *pat_off, *txt_off;
  int32_t k, W, Ov, want_cigar;
  int32_t *score;
  int8_t *status;
  uint32_t *runs;
  const int64_t *slot_off;
  int32_t *nruns;
  int64_t *stats;
  int64_t next;
  int32_t fail;
  pthread_mutex_t mu;
} genasm_job;

static void *genasm_worker(void *arg) {
  genasm_job *J = (genasm_job *)arg;
  for (;;) {
    pthread_mutex_lock(&J->mu);
    const int64_t b = J->next;
    J->next += 16;
    pthread_mutex_unlock(&J->mu);
    if (b >= J->n) return NULL;
    const int64_t e = b + 16 < J->n ? b + 16 : J->n;
    for (int64_t q = b; q < e; ++q) {
      const int32_t m = (int32_t)(J->pat_off[q + 1] - J->pat_off[q]);
      const int32_t n = (int32_t)(J->txt_off[q + 1] - J->txt_off[q]);
      const int64_t so = J->want_cigar ? J->slot_off[q] : 0;
      const int32_t cap = J->want_cigar ? (int32_t)(J->slot_off[q + 1] - J->slot_off[q]) : 0;
      const int rc = oracle_genasm(J->pat + J->pat_off[q], m, J->txt + J->txt_off[q], n, J->k, J->W, J->Ov,
                                   J->want_cigar, J->score + q, J->status + q, J->runs + so, cap, J->nruns + q,
                                   J->stats ? J->stats + 3 * q : NULL);
      if (rc) {
        J->status[q] = -1;
        pthread_mutex_lock(&J->mu);
        J->fail = rc;
        pthread_mutex_unlock(&J->mu);
      }
    }
  }
}

/* stats: NULL, or 3 counters per pair (see oracle_genasm). */
int oracle_genasm_batch(int64_t n, const uint8_t *pat, const int64_t *pat_off, const uint8_t *txt,
                        const int64_t *txt_off, int32_t k, int32_t W, int32_t Ov, int32_t want_cigar,
                        int32_t nthreads, int32_t *score, int8_t *status, uint32_t *runs,
                        const int64_t *slot_off, int32_t *nruns, int64_t *stats) {
  genasm_job J = {n, pat, txt, pat_off, txt_off, k, W, Ov, want_cigar, score, status, runs, slot_off, nruns,
                  stats, 0, 0, PTHREAD_MUTEX_INITIALIZER};
  if (nthreads < 1) nthreads = 1;
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
  if (!th) return -1;
  int started = 0;
  for (int t = 0; t < nthreads; ++t)
    if (pthread_create(&th[started], NULL, genasm_worker, &J) == 0) ++started;
  if (started == 0) genasm_worker(&J);
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  free(th);
  return J.fail;
}
